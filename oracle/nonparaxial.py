"""Gaussian beam beyond the paraxial approximation (oracle, FP64).

The paper motivates tightly focused, nonparaxial beams (Sec. III.A: the
paraxial assumption fails under tight focusing) without writing their fields.
Reading: the Lax-Davis expansion of a linearly polarised vector potential
A = x-hat psi(x, y, z) e^{ikz} (physics convention e^{i(kz - wt)}, vacuum,
c = w = k = 1), psi = psi0 (1 + eps^2 G2 + eps^4 G4), eps = w0/x_R.

The series, written out:
* psi0 = f exp(-f s), f = 1/(1 + i zeta), s = (x^2 + y^2)/w0^2, zeta = z/x_R;
* G2 = f^2 s / 2 - f^3 s^2 / 4 and
  G4 = f^6 s^4 / 32 - f^5 s^3 / 4 + 3 f^4 s^2 / 8: the polynomials in (f, s)
  that make the scaled Helmholtz equation
  lap_perp psi + 4i d_zeta psi + eps^2 d_zeta^2 psi vanish at orders eps^2
  and eps^4, with the homogeneous freedom (zeta-derivatives of psi0, i.e.
  focus and waist redefinitions) fixed by psi = psi0 on the axis (s = 0);
  the pins check the eps^6 residual of the truncated psi;
* E = i A + i grad div A and B = curl A are obtained by symbolic
  differentiation of the full potential in physical coordinates.

The real fields use the pulse convention of ``pulses``: with X the complex
amplitude normalised by i w A0, a field is Re{conj(X) Gamma e^{i(theta + Phi)}},
so that the leading E_p is Re{conj(psi0) Gamma e^{i(theta + Phi)}} like the
paraxial Gaussian.
"""
from functools import lru_cache

import numpy as np
import sympy as sp

from . import pulses as _pulses


def series():
    """(G2, G4) as sympy polynomials in the symbols F (= f) and S (= s)."""
    F, S = sp.symbols("F S")
    G2 = F ** 2 * S / 2 - F ** 3 * S ** 2 / 4
    G4 = F ** 6 * S ** 4 / 32 - F ** 5 * S ** 3 / 4 + sp.Rational(3, 8) * F ** 4 * S ** 2
    return G2, G4


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
