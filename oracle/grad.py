"""Reference gradients of gridless observables (oracle, FP64).

The observable of a gridless run is L = sum_p wu_p . u_p(final) + wp_p proxy_p,
with the run advanced by ``pic.gridless_step``.  Its derivative with respect
to a pulse parameter is taken here by central differences of the FP64
trajectory, Richardson-extrapolated: with D(h) = (L(th + h) - L(th - h))/(2h),
    g = (4 D(h/2) - D(h)) / 3,
whose error is O(h^4) plus FP64 rounding ~ eps |L| / h.
"""
import numpy as np

from . import pic, pulses, units

L = units.LAMBDA


def run_gridless(prm, X0, u0, q_over_m, t0, dt, n_steps):
    """FP64 trajectory; prm in lambda units, X0 (3, N) lab positions in lambda,
    t0, dt in lambda/c.  Returns (X, u, proxy) at the end (internal units for X)."""
    P = pulses.Pulse(prm)
    X = np.array(X0, dtype=float) * L
    u = np.array(u0, dtype=float)
    proxy = np.zeros(u.shape[1])
    t = t0 * L
    for n in range(n_steps):
        X, u, dp = pic.gridless_step(t0 * L + n * dt * L, dt * L, X, u, q_over_m, P, with_proxy=True)
        proxy += dp
    return X, u, proxy


def observable(prm, X0, u0, q_over_m, t0, dt, n_steps, wu, wp):
    _, u, proxy = run_gridless(prm, X0, u0, q_over_m, t0, dt, n_steps)
    return float(np.sum(wu * u) + np.sum(wp * proxy))


def gradient(prm, name, X0, u0, q_over_m, t0, dt, n_steps, wu, wp, rel_h=1e-3):
    """dL/d(prm[name]) by Richardson-extrapolated central differences.

    Returns (g, g_h, g_h2): the extrapolated value and the two central
    differences it combines (their gap measures the truncation error)."""
    base = float(prm[name])
    h = rel_h * max(abs(base), 1.0)

    def Lof(v):
        q = dict(prm)
        q[name] = v
        return observable(q, X0, u0, q_over_m, t0, dt, n_steps, wu, wp)

    d1 = (Lof(base + h) - Lof(base - h)) / (2 * h)
    d2 = (Lof(base + h / 2) - Lof(base - h / 2)) / h
    return (4 * d2 - d1) / 3, d1, d2
