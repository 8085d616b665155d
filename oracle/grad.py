"""Reference gradients of gridless observables (oracle, FP64).

The observable of a gridless run is L = sum_p wu_p . u_p(final) + wp_p proxy_p,
with the run advanced by ``pic.gridless_step``.  Its derivative with respect
to a pulse parameter is taken here by central differences of the FP64
trajectory, Richardson-extrapolated: with D(h) = (L(th + h) - L(th - h))/(2h),
    g = (4 D(h/2) - D(h)) / 3,
whose error is O(h^4) plus FP64 rounding ~ eps |L| / h.

Gridded runs have two references: the frozen-grid one (one species pushed
through the E2, B2 a nominal run recorded) and the fully coupled one (the
whole loop, every species, rerun at each perturbed parameter).
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


# ----------------------------------------------------------------------------
# Gridded runs, frozen-grid reading: E2, B2 are the fields a nominal
# self-consistent run produced at the start of each step, taken as an external
# field; the gradient is that of the particles pushed through them.
# ----------------------------------------------------------------------------

def record_gridded_run(grid, species, prm, n_steps, pulse_on_grid=False):
    """Nominal run of the full loop (pic.step) from the given state.  Returns
    [(E2, B2, t)] at the start of every step; grid and species end at the
    final state."""
    P = pulses.Pulse(prm)
    recs = []
    for _ in range(n_steps):
        recs.append(([e.copy() for e in grid.E], [b.copy() for b in grid.B], grid.t))
        pic.step(grid, species, P, pulse_on_grid=pulse_on_grid)
    return recs


def frozen_run(prm, grid, recs, sp0, pulse_on_grid=False, with_proxy=False):
    """One species pushed through the recorded fields (no deposit, no field
    update).  ``grid`` supplies the geometry; returns the final (pos, u), and
    the emission proxy accumulated from zero with ``with_proxy``."""
    P = pulses.Pulse(prm)
    sp = pic.Species(sp0.q, sp0.m, sp0.pos, sp0.u, sp0.w)
    proxy = np.zeros(sp.u.shape[1])
    saved = grid.E, grid.B, grid.t
    try:
        for E, B, t in recs:
            grid.E, grid.B, grid.t = E, B, t
            u_half, Ep, Bp = pic.push_species(grid, sp, P, pulse_on_grid=pulse_on_grid, with_fields=True)
            proxy = proxy + pic.emission_proxy(sp.u, u_half, Ep, Bp, grid.dt)
            new = pic.move(grid, sp.pos, u_half)
            sp.u = u_half
            sp.pos = pic.wrap(grid, new)
    finally:
        grid.E, grid.B, grid.t = saved
    return (sp.pos, sp.u, proxy) if with_proxy else (sp.pos, sp.u)


def frozen_gradient(prm, name, grid, recs, sp0, wu, rel_h=1e-6, pulse_on_grid=False, wp=None):
    """dL/d(prm[name]), L = sum wu . u_final (+ sum wp proxy_final), through the recorded fields:
    Richardson-extrapolated central differences as in ``gradient``.

    L has jumps: a particle that crosses the periodic boundary one step
    earlier or later samples the (non-periodic) pulse a box length away.  On
    small boxes they lie within 1e-4 relative of the nominal parameters, so
    the step is kept small; at 1e-6 the round-off of L stays near 1e-10
    relative."""
    base = float(prm[name])
    h = rel_h * max(abs(base), 1.0)

    def Lof(v):
        q = dict(prm)
        q[name] = v
        if wp is None:
            return float(np.sum(wu * frozen_run(q, grid, recs, sp0, pulse_on_grid)[1]))
        _, u, pr = frozen_run(q, grid, recs, sp0, pulse_on_grid, with_proxy=True)
        return float(np.sum(wu * u) + np.sum(wp * pr))

    d1 = (Lof(base + h) - Lof(base - h)) / (2 * h)
    d2 = (Lof(base + h / 2) - Lof(base - h / 2)) / h
    return (4 * d2 - d1) / 3, d1, d2


# ----------------------------------------------------------------------------
# Gridded runs, fully coupled: the parameters act on every species through
# E1, B1 and, through the deposited current and the Yee update, on E2, B2.
# ----------------------------------------------------------------------------

def _clone(grid, species):
    g = pic.Grid(grid.dim, grid.n, grid.dx, grid.dt, grid.x_min, t0=grid.t, open_x=grid.open_x)
    g.E = [e.copy() for e in grid.E]
    g.B = [b.copy() for b in grid.B]
    sps = [pic.Species(sp.q, sp.m, sp.pos, sp.u, sp.w, proxy=None if sp.proxy is None else sp.proxy)
           for sp in species]
    return g, sps


def coupled_run(prm, grid, species, n_steps, sp_index=0, with_proxy=False):
    """The full loop (pic.step: push, deposit, Yee) for n_steps from copies of
    ``grid`` and ``species`` (left unchanged).  Returns the final u of species
    ``sp_index`` and, with ``with_proxy``, its emission proxy accumulated from
    zero."""
    P = pulses.Pulse(prm)
    g, sps = _clone(grid, species)
    if with_proxy:
        sps[sp_index].proxy = np.zeros(sps[sp_index].u.shape[1])
    for _ in range(n_steps):
        pic.step(g, sps, P)
    sp = sps[sp_index]
    return (sp.u, sp.proxy) if with_proxy else sp.u


def coupled_gradient(prm, name, grid, species, n_steps, wu, sp_index=0, rel_h=1e-6, wp=None):
    """dL/d(prm[name]) through the whole self-consistent run, L = sum wu . u_final
    (+ sum wp proxy_final) of species ``sp_index``: Richardson-extrapolated
    central differences as in ``frozen_gradient`` (the same jumps apply)."""
    base = float(prm[name])
    h = rel_h * max(abs(base), 1.0)

    def Lof(v):
        q = dict(prm)
        q[name] = v
        if wp is None:
            return float(np.sum(wu * coupled_run(q, grid, species, n_steps, sp_index)))
        u, pr = coupled_run(q, grid, species, n_steps, sp_index, with_proxy=True)
        return float(np.sum(wu * u) + np.sum(wp * pr))

    d1 = (Lof(base + h) - Lof(base - h)) / (2 * h)
    d2 = (Lof(base + h / 2) - Lof(base - h / 2)) / h
    return (4 * d2 - d1) / 3, d1, d2
