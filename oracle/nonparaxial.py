"""Gaussian beam beyond the paraxial approximation (oracle, FP64).

The paper motivates tightly focused, nonparaxial beams (Sec. III.A: the
paraxial assumption fails under tight focusing) without writing their fields.
Reading: the Lax-Davis expansion of a linearly polarised vector potential
A = x-hat psi(x, y, z) e^{ikz} (physics convention e^{i(kz - wt)}, vacuum,
c = w = k = 1), psi = psi0 (1 + eps^2 G2 + eps^4 G4), eps = w0/x_R.

This module derives the series by itself:
* psi0 = f exp(-f s), f = 1/(1 + i zeta), s = (x^2 + y^2)/w0^2, zeta = z/x_R;
* G2, G4 are polynomials in (f, s) found by making the scaled Helmholtz
  equation lap_perp psi + 4i d_zeta psi + eps^2 d_zeta^2 psi vanish order by
  order, matched numerically on random points and rationalised;
* the homogeneous freedom (zeta-derivatives of psi0, i.e. focus and waist
  redefinitions) is removed by requiring psi = psi0 on the axis;
* E = i A + i grad div A and B = curl A are obtained by symbolic
  differentiation of the full potential in physical coordinates.

The real fields use the pulse convention of ``pulses``: with X the complex
amplitude normalised by i w A0, a field is Re{conj(X) Gamma e^{i(theta + Phi)}},
so that the leading E_p is Re{conj(psi0) Gamma e^{i(theta + Phi)}} like the
paraxial Gaussian.
"""
from fractions import Fraction
from functools import lru_cache

import numpy as np
import sympy as sp

from . import pulses as _pulses


def _lin_solve_rational(A, b):
    """Least-squares solve and rationalise (coefficients are small rationals)."""
    x, *_ = np.linalg.lstsq(A, b, rcond=None)
    out = []
    for v in x:
        re = Fraction(float(v.real)).limit_denominator(512)
        im = Fraction(float(v.imag)).limit_denominator(512)
        out.append(sp.Rational(re.numerator, re.denominator)
                   + sp.I * sp.Rational(im.numerator, im.denominator))
    return out


@lru_cache(maxsize=1)
def series():
    """(G2, G4) as sympy expressions in (f, s) symbols F, S."""
    xi, eta, zeta = sp.symbols("xi eta zeta", real=True)
    F, S = sp.symbols("F S")
    f = 1 / (1 + sp.I * zeta)
    s = xi ** 2 + eta ** 2
    psi0 = f * sp.exp(-f * s)

    def helm(g):   # lap_perp + 4 i d_zeta
        return sp.diff(g, xi, 2) + sp.diff(g, eta, 2) + 4 * sp.I * sp.diff(g, zeta)

    rng = np.random.default_rng(12345)
    pts = np.stack([rng.uniform(-1.5, 1.5, 120), rng.uniform(-1.5, 1.5, 120),
                    rng.uniform(-2.0, 2.0, 120)], axis=1)
    Gs = [sp.Integer(1)]
    for n in (1, 2):
        monos = [(a, b) for a in range(1, 4 * n + 2) for b in range(0, 2 * n + 1)]
        cols = []
        for (a, b) in monos:
            e = helm(f ** a * s ** b * psi0) / psi0
            fn = sp.lambdify((xi, eta, zeta), e, "numpy")
            cols.append(np.array([complex(fn(*p)) for p in pts]))
        rhs_e = sp.diff(Gs[-1].subs({F: f, S: s}) * psi0, zeta, 2) / psi0
        fr = sp.lambdify((xi, eta, zeta), rhs_e, "numpy")
        rhs = -np.array([complex(fr(*p)) for p in pts])
        A = np.stack(cols, axis=1)
        # on-axis condition: sum_a c_{a,0} f^a = 0 for every zeta
        zs = np.linspace(-2, 2, 9)
        rows = np.zeros((zs.size, len(monos)), dtype=complex)
        for j, (a, b) in enumerate(monos):
            if b == 0:
                rows[:, j] = (1.0 / (1.0 + 1j * zs)) ** a
        A = np.vstack([A, rows * 10.0])
        rhs = np.concatenate([rhs, np.zeros(zs.size)])
        c = _lin_solve_rational(A, rhs)
        Gn = sp.expand(sum(ci * F ** a * S ** b for ci, (a, b) in zip(c, monos)))
        Gs.append(Gn)
    return Gs[1], Gs[2]


@lru_cache(maxsize=4)
def _field_functions():
    """Lambdified complex amplitudes X (normalised by i A0) of E and B in the
    physics frame (x = polarisation, y, z = propagation), as functions of
    (x, y, z, w0, e2w, e4w) with e2w, e4w the truncation weights of psi."""
    x, y, z, w0 = sp.symbols("x y z w0", real=True)
    e2w, e4w = sp.symbols("e2w e4w", real=True)
    F, S = sp.symbols("F S")
    G2, G4 = series()
    xr = w0 ** 2 / 2              # k w0^2 / 2 with k = 1
    zeta = z / xr
    f = 1 / (1 + sp.I * zeta)
    s = (x ** 2 + y ** 2) / w0 ** 2
    G = 1 + e2w * G2.subs({F: f, S: s}) + e4w * G4.subs({F: f, S: s})
    A = G * f * sp.exp(-f * s) * sp.exp(sp.I * z)
    divA = sp.diff(A, x)
    E = [sp.I * (A + sp.diff(divA, x)), sp.I * sp.diff(divA, y), sp.I * sp.diff(divA, z)]
    B = [sp.Integer(0) * A, sp.diff(A, z), -sp.diff(A, y)]
    carrier = sp.exp(-sp.I * z) / sp.I
    out = [sp.lambdify((x, y, z, w0, e2w, e4w), sp.expand(comp * carrier), "numpy", cse=True) for comp in E + B]
    return out


def fields(P, t, X, Y, Z):
    """E1, B1 of the nonparaxial Gaussian at lab points (internal units)."""
    if abs(P.v_phi - 1.0) > 0 or abs(P.b_over_e - 1.0) > 0:
        raise ValueError("the nonparaxial Gaussian is a vacuum solution (use DISP_VACUUM)")
    gam, phi = _pulses._envelope(P, t, X)
    theta = _pulses._carrier(P, t, X)
    p, q = _pulses._transverse(P, Y, Z)
    zz = X - P.x_f
    e2w = (P.w0 / P.x_r) ** 2 if P.np_order >= 2 else 0.0
    e4w = (P.w0 / P.x_r) ** 4 if P.np_order >= 4 else 0.0
    fn = _field_functions()
    vals = [np.broadcast_to(np.asarray(g(p, q, zz, P.w0, e2w, e4w), dtype=complex), np.shape(X))
            for g in fn]
    V = gam * np.exp(1j * (theta + phi))
    re = [np.real(np.conj(v) * V) for v in vals]
    # physics frame (x, y, z) = pulse frame (p, q, propagation)
    e_p, e_q, e_x = re[0], re[1], re[2]
    b_p, b_q, b_x = re[3], re[4], re[5]
    return _pulses.to_lab(P, (e_x, e_p, e_q), (b_x, b_p, b_q))
