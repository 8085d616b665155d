"""Analytic vacuum fields E1, B1 (oracle, FP64).

The field split of Eqs. (3)-(4): E = E1 + E2, B = B1 + B2, where (E1, B1) is
an approximate closed-form vacuum solution (the laser) and (E2, B2) is the
plasma response carried on the grid.  This module evaluates (E1, B1) at
arbitrary points and one time, in the normalised units of ``units``.

Pulse frame: the pulse propagates along +x; its primary electric field lies
along the polarisation axis p and its primary magnetic field along
q = x-hat cross p-hat (Sec. II.A takes k || x, E || y, B || z).
``pol = 0`` puts p along y (q along z); ``pol = 1`` puts p along z (q along
-y), the in-plane choice for an (x, z) grid.

Parameters arrive as a dict in lambda units (lambda = 1, c = 1) and are
converted here with the factor 2*pi of ``units``:

    type        'plane' | 'gauss' | 'lg' | 'ff' | 'gauss_np'
    a0          peak field amplitude (Sec. II.A, Fig. 3 caption)
    tau         full (zero-to-zero) duration of the sin^2 field envelope
    t_ref,x_ref the envelope peak passes x_ref at time t_ref
    phi0        carrier phase at (t_ref, x_ref)  ("initial phase at a
                specified reference position", Sec. II.B)
    chirp       fractional frequency sweep across tau (Phi of Eq. (15))
    x_f, w0     focal position and waist (Eqs. (21)-(23))
    y_c, z_c    transverse position of the beam axis
    q_slice     value of the ignorable coordinate y on an (x, z) grid
    d_f         focusing dimensionality D of Eq. (21): 2 or 3
    lg_l, lg_p  Laguerre-Gaussian azimuthal and radial indices
    pol         0 (p = y) or 1 (p = z)
    beta_f, x0_ff, t0_ff   flying focus: focal velocity / c, focus at x0_ff
                           at time t0_ff (Sec. III.C)
    dispersion  units.DISP_PAPER2 | DISP_EXACT | DISP_VACUUM | DISP_PLASMA
    dx_prop, dt cell size along x and time step, lambda units (fix the
                numerical v_phi, v_g, B0/E0 of Eqs. (10)-(14))
    np_order    0 or 4: order in eps = w0/x_R of the nonparaxial Gaussian
    envelope    'sin2' (default) or 'sgauss': super-Gaussian of order
                sg_order whose intensity full width at half maximum is
                fwhm (lambda/c), centred in the support [0, tau]
    wp2, zeta   DISP_PLASMA (Sec. IV): omega_p^2/omega^2 of the density the
                analytic current J1 represents, and the factor zeta of the
                plasma's discrete response (default 1)
    fd          DISP_PLASMA: keep the lowest-order finite-duration
                corrections of B1 and J1 (default True)
"""
import math

import numpy as np

from . import units

TYPES = ("plane", "gauss", "lg", "ff", "gauss_np")


class Pulse:
    """Derived constants of one pulse, internal units (Sec. II.A, Sec. III)."""

    def __init__(self, prm):
        L = units.LAMBDA
        self.kind = prm["type"]
        if self.kind not in TYPES:
            raise ValueError("unknown pulse type %r" % (self.kind,))
        self.a0 = float(prm.get("a0", 1.0))
        self.tau = float(prm.get("tau", 10.0)) * L
        self.t_ref = float(prm.get("t_ref", 0.0)) * L
        self.x_ref = float(prm.get("x_ref", 0.0)) * L
        self.phi0 = float(prm.get("phi0", 0.0))
        self.chirp = float(prm.get("chirp", 0.0))
        self.x_f = float(prm.get("x_f", 0.0)) * L
        self.w0 = float(prm.get("w0", 5.0)) * L
        self.y_c = float(prm.get("y_c", 0.0)) * L
        self.z_c = float(prm.get("z_c", 0.0)) * L
        self.q_slice = float(prm.get("q_slice", 0.0)) * L
        self.d_f = int(prm.get("d_f", 3))
        self.lg_l = int(prm.get("lg_l", 0))
        self.lg_p = int(prm.get("lg_p", 0))
        self.pol = int(prm.get("pol", 0))
        self.beta_f = float(prm.get("beta_f", 0.0))
        self.x0_ff = float(prm.get("x0_ff", 0.0)) * L
        self.t0_ff = float(prm.get("t0_ff", 0.0)) * L
        self.np_order = int(prm.get("np_order", 4))
        mode = int(prm.get("dispersion", units.DISP_PAPER2))
        dx = float(prm.get("dx_prop", 0.05)) * L
        dt = float(prm.get("dt", 0.0)) * L
        if mode != units.DISP_VACUUM and dt <= 0.0:
            raise ValueError("grid dispersion modes need dx_prop and dt")
        self.wp2 = float(prm.get("wp2", 0.0))
        self.zeta = float(prm.get("zeta", 1.0))
        self.fd = bool(prm.get("fd", True))
        self.current = mode == units.DISP_PLASMA
        if self.current and self.kind == "gauss_np":
            raise ValueError("the nonparaxial Gaussian is a vacuum field")
        self.v_phi, self.v_g, self.b_over_e, self.k = units.dispersion(mode, dx, dt, self.wp2, self.zeta)
        self.omega = 1.0
        # Rayleigh range x_R = k w0^2 / 2 with k = omega / v_phi (Eq. (23)).
        self.x_r = self.k * self.w0 ** 2 / 2.0
        # Linear chirp: instantaneous frequency omega + b (eta - tau/2), so that
        # the sweep across the envelope is chirp * omega.
        self.b = self.chirp * self.omega / self.tau
        self.lg_norm = _lg_peak_norm(abs(self.lg_l), self.lg_p) if self.kind == "lg" else 1.0
        # Temporal envelope: sin^2, or the super-Gaussian the paper's runs use
        # (Sec. II.B), exp(-((eta - tau/2)/tau_g)^(2g)); tau_g is fixed by the
        # intensity FWHM: Gamma^2 = 1/2 at (eta - tau/2)/tau_g = (ln 2 / 2)^(1/2g).
        self.envelope = prm.get("envelope", "sin2")
        if self.envelope not in ("sin2", "sgauss"):
            raise ValueError("unknown envelope %r" % (self.envelope,))
        self.sg_order = int(prm.get("sg_order", 4))
        self.fwhm = float(prm.get("fwhm", 0.0)) * L
        if self.envelope == "sgauss":
            if self.sg_order < 1 or not self.fwhm > 0.0:
                raise ValueError("the super-Gaussian envelope needs sg_order >= 1 and fwhm > 0")
            self.tau_g = self.fwhm / (2.0 * (math.log(2.0) / 2.0) ** (1.0 / (2 * self.sg_order)))
        if self.kind == "lg" and self.d_f != 3:
            raise ValueError("Laguerre-Gaussian modes need d_f = 3")


def _laguerre(n, alpha, x):
    """Generalised Laguerre polynomial L_n^alpha(x) by its three-term recurrence."""
    l_prev = np.ones_like(x)
    if n == 0:
        return l_prev
    l_cur = 1.0 + alpha - x
    for m in range(1, n):
        l_next = ((2 * m + 1 + alpha - x) * l_cur - (m + alpha) * l_prev) / (m + 1)
        l_prev, l_cur = l_cur, l_next
    return l_cur


def _laguerre_deriv(n, alpha, x):
    """d/dx L_n^alpha(x) = -L_{n-1}^{alpha+1}(x)."""
    if n == 0:
        return np.zeros_like(x)
    return -_laguerre(n - 1, alpha + 1, x)


def _lg_peak_norm(l_abs, p):
    """Scale so that the peak |F| of an LG mode at focus is one.

    a0 is the peak field (reading of Sec. II.A: a0 = |e|E0/(m c omega)); at
    focus |F| is (sqrt(2) r/w0)^|l| |L_p^|l|(2 r^2/w0^2)| exp(-r^2/w0^2), whose
    maximum over r is bracketed on a dense grid in x = 2 r^2 / w0^2 and then
    refined by a bounded scalar minimisation.
    """
    from scipy.optimize import minimize_scalar

    def prof(x):
        return x ** (l_abs / 2.0) * np.abs(_laguerre(p, l_abs, np.asarray(x, dtype=float))) * np.exp(-x / 2.0)
    x = np.linspace(0.0, 60.0, 60001)
    i = int(np.argmax(prof(x)))
    lo, hi = x[max(i - 1, 0)], x[min(i + 1, x.size - 1)]
    if hi <= lo:
        return 1.0 / float(prof(x[i]))
    res = minimize_scalar(lambda v: -float(prof(v)), bounds=(lo, hi), method="bounded",
                          options={"xatol": 1e-13})
    return 1.0 / max(float(prof(res.x)), float(prof(x[i])))


def _envelope(P, t, X):
    """Envelope Gamma (sin^2 or super-Gaussian) and chirp phase Phi of Eq. (15).

    eta = (t - t_ref) - (x - x_ref)/v_g + tau/2 is the envelope argument
    t - x/v_g shifted so that the support is 0 <= eta <= tau and the peak
    passes x_ref at t_ref.
    """
    eta = (t - P.t_ref) - (X - P.x_ref) / P.v_g + P.tau / 2.0
    inside = (eta >= 0.0) & (eta <= P.tau)
    if P.envelope == "sgauss":
        prof = np.exp(-((eta - P.tau / 2.0) / P.tau_g) ** (2 * P.sg_order))
    else:
        prof = np.sin(math.pi * eta / P.tau) ** 2
    gam = np.where(inside, P.a0 * prof, 0.0)
    phi = 0.5 * P.b * (eta - P.tau / 2.0) ** 2
    return gam, phi


def _envelope_rates(P, t, X):
    """Time derivatives at fixed x of the envelope and the chirp phase, as
    Gamma'/Gamma, Gamma''/Gamma, Phi', Phi'' (zero outside the support)."""
    eta = (t - P.t_ref) - (X - P.x_ref) / P.v_g + P.tau / 2.0
    inside = (eta > 0.0) & (eta < P.tau)
    if P.envelope == "sgauss":
        g = P.sg_order
        x = (eta - P.tau / 2.0) / P.tau_g
        g1 = -2.0 * g * x ** (2 * g - 1) / P.tau_g
        g2 = g1 * g1 - 2.0 * g * (2 * g - 1) * x ** (2 * g - 2) / P.tau_g ** 2
    else:
        a = math.pi / P.tau
        sn = np.where(inside, np.sin(a * eta), 1.0)
        cs = np.cos(a * eta)
        g1 = 2.0 * a * cs / sn
        g2 = 2.0 * a * a * (cs * cs - sn * sn) / (sn * sn)
    p1 = P.b * (eta - P.tau / 2.0)
    p2 = np.full_like(eta, P.b)
    zero = np.zeros_like(eta)
    return (np.where(inside, g1, zero), np.where(inside, g2, zero), np.where(inside, p1, zero),
            np.where(inside, p2, zero))


def fd_factor(P, t, X, delta):
    """Lowest-order finite-duration correction (Sec. IV) as a complex factor
    A exp(i psi) on Gamma exp(i(Theta + Phi)), for a field whose spectrum is
    the envelope's times 1 + delta sum_n (i/omega)^n d^n/dt^n:
        A   = 1 - delta Gamma''/(w^2 Gamma) + (delta Gamma'/(w Gamma))^2 / 2
                - delta Phi'/w + delta Phi'^2 / w^2,
        psi = delta Gamma'/(w Gamma) - delta Phi''/w^2 - 2 delta (Gamma'/Gamma) Phi'/w^2.
    delta = 1 - v_phi/v_g gives B1 (the B_z form of Sec. IV), delta = 1 the
    integral of E1 that J1 carries."""
    g1, g2, p1, p2 = _envelope_rates(P, t, X)
    w = P.omega
    amp = 1.0 - delta * g2 / w ** 2 + 0.5 * (delta * g1 / w) ** 2 - delta * p1 / w + delta * p1 ** 2 / w ** 2
    psi = delta * g1 / w - delta * p2 / w ** 2 - 2.0 * delta * g1 * p1 / w ** 2
    return amp * np.exp(1j * psi)


def _carrier(P, t, X):
    """Carrier phase omega (t - x/v_phi) of Eq. (15), referenced to (t_ref, x_ref)."""
    return P.omega * (t - P.t_ref) - P.k * (X - P.x_ref) + P.phi0


def _transverse(P, Y, Z):
    """Pulse-frame transverse coordinates (p, q) of lab points."""
    if P.pol == 0:
        return Y - P.y_c, Z - P.z_c
    return Z - P.z_c, -(Y - P.y_c)


def _gauss_profile(P, s, p, q, k_c, x_r, gouy_extra=0.0):
    """Paraxial Gaussian F of Eqs. (21)-(23) and its transverse derivatives.

    s = x_f - x is the distance to focus; ``k_c`` is the wavenumber that
    multiplies the curvature term and ``x_r`` the Rayleigh range (both are
    replaced for the flying focus).  Returns (F, dF/dp, dF/dq) as complex
    arrays.  For d_f = 2 the beam is focused only in the (x, z) plane, so
    r is the lab z offset; for d_f = 3, r^2 = p^2 + q^2.
    """
    w0 = P.w0
    w2 = w0 ** 2 * (1.0 + s ** 2 / x_r ** 2)
    inv_r = s / (s ** 2 + x_r ** 2)               # 1/R without the focal singularity
    if P.d_f == 3:
        r2 = p ** 2 + q ** 2
        dr2_dp, dr2_dq = 2.0 * p, 2.0 * q
    else:
        if P.pol == 1:   # p is the in-plane transverse axis z
            r2, dr2_dp, dr2_dq = p ** 2, 2.0 * p, 0.0 * q
        else:            # q is the in-plane transverse axis z
            r2, dr2_dp, dr2_dq = q ** 2, 0.0 * p, 2.0 * q
    half_d = (P.d_f - 1) / 2.0
    gouy = (half_d + gouy_extra) * np.arctan(s / x_r)
    amp = (w0 ** 2 / w2) ** (half_d / 2.0) * np.exp(-r2 / w2)
    phase = k_c * r2 * inv_r / 2.0 - gouy
    F = amp * np.exp(1j * phase)
    dlog = -1.0 / w2 + 1j * k_c * inv_r / 2.0     # d(log F)/d(r^2)
    return F, F * dlog * dr2_dp, F * dlog * dr2_dq, w2


def _profile(P, t, X, Y, Z):
    """Complex transverse profile F and dF/dp, dF/dq at lab points."""
    p, q = _transverse(P, Y, Z)
    if P.kind == "plane":
        one = np.ones_like(X, dtype=complex)
        return one, 0.0 * one, 0.0 * one
    if P.kind == "gauss":
        F, Fp, Fq, _ = _gauss_profile(P, P.x_f - X, p, q, P.k, P.x_r)
        return F, Fp, Fq
    if P.kind == "ff":
        # Sec. III.C: Eq. (21) with x_R -> (1 - beta_f) x_R and x_f - x -> xi_0 - xi,
        # xi = x - v_f t, xi_0 = x_0 - v_f t_0.  The curvature term carries
        # k' = (1 - beta_f) k so that F solves Eq. (26) exactly.
        s = P.x0_ff + P.beta_f * (t - P.t0_ff) - X
        one_m_b = 1.0 - P.beta_f
        F, Fp, Fq, _ = _gauss_profile(P, s, p, q, one_m_b * P.k, one_m_b * P.x_r)
        return F, Fp, Fq
    if P.kind == "lg":
        l_abs, n = abs(P.lg_l), P.lg_p
        sig = 1.0 if P.lg_l >= 0 else -1.0
        G, Gp, Gq, w2 = _gauss_profile(P, P.x_f - X, p, q, P.k, P.x_r,
                                       gouy_extra=float(2 * n + l_abs))
        c = P.lg_norm * (2.0 / w2) ** (l_abs / 2.0)
        pq = p + 1j * sig * q
        A = c * pq ** l_abs
        if l_abs > 0:
            Ap = c * l_abs * pq ** (l_abs - 1)
            Aq = 1j * sig * Ap
        else:
            Ap = Aq = 0.0 * pq
        rho = 2.0 * (p ** 2 + q ** 2) / w2
        Lg = _laguerre(n, l_abs, rho)
        dL = _laguerre_deriv(n, l_abs, rho)
        F = A * Lg * G
        Fp = Ap * Lg * G + A * dL * (4.0 * p / w2) * G + A * Lg * Gp
        Fq = Aq * Lg * G + A * dL * (4.0 * q / w2) * G + A * Lg * Gq
        return F, Fp, Fq
    raise ValueError("profile not defined for %r" % P.kind)


def analytic_fields(P, t, X, Y, Z):
    """E1, B1 at lab points (X, Y, Z) and time t, internal units.

    Primary components (Eq. (15) times F, Sec. III.A):
        E_p = Re{Gamma F exp(i(theta + Phi))},   B_q = (B0/E0) E_p   (Eq. (17)).
    Secondary components from the divergence relations of Sec. III.A, with
    derivatives acting on F only:
        E_x = Re{-i (v_phi/omega) dF/dp Gamma exp(i(theta + Phi))}
        B_x = Re{-i (c/omega) (B0/E0) dF/dq Gamma exp(i(theta + Phi))}.
    Returns (E, B), each of shape (3,) + X.shape, lab components (x, y, z).
    """
    X = np.asarray(X, dtype=float)
    Y = np.broadcast_to(np.asarray(Y, dtype=float), X.shape)
    Z = np.broadcast_to(np.asarray(Z, dtype=float), X.shape)
    if P.kind == "gauss_np":
        from . import nonparaxial
        return nonparaxial.fields(P, t, X, Y, Z)
    gam, phi = _envelope(P, t, X)
    theta = _carrier(P, t, X)
    F, Fp, Fq = _profile(P, t, X, Y, Z)
    carrier = gam * np.exp(1j * (theta + phi))
    e_p = np.real(F * carrier)
    e_x = np.real(-1j * (P.v_phi / P.omega) * Fp * carrier)
    # B1: Eq. (17) in vacuum; with an analytic current the finite-duration
    # correction of Sec. IV (delta = 1 - v_phi/v_g), unless switched off
    cb = carrier * fd_factor(P, t, X, 1.0 - P.v_phi / P.v_g) if (P.current and P.fd) else carrier
    b_q = P.b_over_e * np.real(F * cb)
    b_x = np.real(-1j * (1.0 / P.omega) * P.b_over_e * Fq * cb)
    zero = np.zeros_like(e_p)
    return to_lab(P, (e_x, e_p, zero), (b_x, zero, b_q))


def analytic_current(P, t, X, Y, Z):
    """Analytic current J1 of Sec. IV at lab points and time t (internal units,
    dJ1/dt = omega_p^2 zeta E1 with 4 pi absorbed): each component of E1 =
    Re{G Gamma e^{i(Theta + Phi)}} gives
        J1 = (wp2 zeta / omega) Re{-i G Gamma e^{i(Theta + Phi)} C},
    C the finite-duration factor with delta = 1 (1 with ``fd`` off).  The
    transverse factor G is held fixed over the integral (slowly varying).
    Returns J (3,) + X.shape, lab components; zero without DISP_PLASMA."""
    X = np.asarray(X, dtype=float)
    Y = np.broadcast_to(np.asarray(Y, dtype=float), X.shape)
    Z = np.broadcast_to(np.asarray(Z, dtype=float), X.shape)
    if not P.current:
        return np.zeros((3,) + X.shape)
    gam, phi = _envelope(P, t, X)
    theta = _carrier(P, t, X)
    F, Fp, Fq = _profile(P, t, X, Y, Z)
    carrier = gam * np.exp(1j * (theta + phi))
    if P.fd:
        carrier = carrier * fd_factor(P, t, X, 1.0)
    pre = P.wp2 * P.zeta / P.omega
    j_p = pre * np.real(-1j * F * carrier)
    j_x = pre * np.real(-1j * (-1j * (P.v_phi / P.omega) * Fp) * carrier)
    zero = np.zeros_like(j_p)
    return to_lab(P, (j_x, j_p, zero), (zero, zero, zero))[0]


def to_lab(P, e_xpq, b_xpq):
    """Rotate pulse-frame (x, p, q) components to lab (x, y, z)."""
    ex, ep, eq = e_xpq
    bx, bp, bq = b_xpq
    if P.pol == 0:      # p = y, q = z
        return np.stack([ex, ep, eq]), np.stack([bx, bp, bq])
    # p = z, q = -y
    return np.stack([ex, -eq, ep]), np.stack([bx, -bq, bp])
