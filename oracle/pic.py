"""The modified PIC step (oracle, FP64, NumPy).

Fig. 1 of the paper: the analytic fields E1, B1 are added to the internally
advanced fields E2, B2, the total field is interpolated to the particles and
used for the particle push, and the particle current drives the internal
field update of E2, B2 only (Eq. (4)).  The paper evaluates E1, B1 on the
grid before interpolation (``pulse_on_grid=True`` here: each component is
sampled at its own staggered node and added to E2, B2 before the gather);
the default evaluates them at the particle position, and only E2, B2 are
interpolated.

Grid conventions (internal units, periodic in every direction):
* arrays are indexed [k, j, i] = (z, y, x); 2-D (x, z) grids have ny = 1 and
  no y derivatives or y motion;
* Yee staggering (Eqs. (7)-(9) generalised to three dimensions):
  Ex (i+1/2, j, k), Ey (i, j+1/2, k), Ez (i, j, k+1/2),
  Bx (i, j+1/2, k+1/2), By (i+1/2, j, k+1/2), Bz (i+1/2, j+1/2, k);
  J components sit with the E components;
* particle positions are in cell units relative to the grid origin, one row
  per axis (x, y, z); the y row is unused on 2-D grids.

Particle shape: quadratic B-spline ("second-order", Sec. II.B: the scaling
runs used second-order current deposition) for both the gather and the
charge-conserving deposition.

Open x ends (``Grid(..., open_x=True)``): the traditional
comparison runs of Fig. demo launch the pulse through an incoming-wave
boundary at x_min (App. B) and let it leave through x_max.  E nodes 0 and
nx - 1 are the boundary nodes; the B nodes at nx - 1/2 lie outside and are
held at zero.  Particles stay periodic: the runs keep plasma away from the
ends.
"""
import math

import numpy as np

from . import pulses as _pulses
from . import units as _units

E_STAGGER = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))
B_STAGGER = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))
_AXIS_OF = {0: 2, 1: 1, 2: 0}   # lab axis -> numpy array axis


class Grid:
    """Internal fields E2, B2 and current J on a periodic Yee grid.

    dim 3: (x, y, z); dim 2: (x, z), the lab y of every node being the
    pulse's slice; dim 1: rows of independent 1-D grids along x (the
    reduced-dimensionality series of Sec. III.B), row k at lab z = x_min[2] +
    k dx[2] and lab y = the pulse's slice.  An inactive axis has no
    derivative, no motion and no stagger; a particle's coordinate on it is
    the (integer) index of its row.  ``open_x``: the x ends are
    incoming/outgoing-wave boundaries for E2, B2 (App. B; on 2-D and 3-D
    grids the boundary update omits the transverse derivatives of B_x, as
    App. B does)."""

    def __init__(self, dim, n, dx, dt, x_min, t0=0.0, open_x=False):
        if dim not in (1, 2, 3):
            raise ValueError("grid dimension must be 1, 2 or 3")
        self.dim = dim
        self.open_x = bool(open_x)
        nx, ny, nz = n
        if dim in (1, 2):
            ny = 1
        self.n = (int(nx), int(ny), int(nz))
        self.dx = tuple(float(d) for d in dx)
        self.dt = float(dt)
        self.x_min = tuple(float(v) for v in x_min)
        self.t = float(t0)
        shape = (self.n[2], self.n[1], self.n[0])
        self.E = [np.zeros(shape) for _ in range(3)]
        self.B = [np.zeros(shape) for _ in range(3)]
        self.J = [np.zeros(shape) for _ in range(3)]

    def active(self, axis):
        return self.dim == 3 or (self.dim == 2 and axis != 1) or axis == 0


class Species:
    """Macroparticles: positions (cell units), momenta u = gamma beta, weights;
    ``proxy`` (per particle, or None) accumulates the emission proxy."""

    def __init__(self, q, m, pos, u, w, proxy=None, ids=None, free=None):
        self.q = float(q)
        self.m = float(m)
        self.pos = np.array(pos, dtype=float, copy=True)
        self.u = np.array(u, dtype=float, copy=True)
        self.w = np.array(w, dtype=float, copy=True)
        self.proxy = None if proxy is None else np.array(proxy, dtype=float, copy=True)
        # particle ids and the ids not in use (moving window bookkeeping)
        self.ids = None if ids is None else np.array(ids, dtype=np.int64, copy=True)
        self.free = np.zeros(0, dtype=np.int64) if free is None else np.sort(np.array(free, dtype=np.int64))


# ----------------------------------------------------------------------------
# Particle shape
# ----------------------------------------------------------------------------

def tsc(d):
    """Quadratic B-spline of a node at distance d (cell units)."""
    a = np.abs(d)
    return np.where(a <= 0.5, 0.75 - a ** 2,
                    np.where(a <= 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def _stencil(xc, stagger):
    """Nodes and weights of the 3-point quadratic stencil on a staggered lattice.

    A component staggered by ``stagger`` cells has nodes at integer + stagger;
    returns the three lattice indices around the nearest node and their
    weights (each of shape (3, N)).
    """
    xs = xc - stagger
    near = np.floor(xs + 0.5)
    offs = np.arange(-1, 2)[:, None]
    nodes = near[None, :] + offs
    return nodes.astype(np.int64), tsc(xs[None, :] - nodes)


def gather(grid, pos):
    """Interpolate E2, B2 to particle positions (quadratic shape, periodic)."""
    out = []
    for comps, stag in ((grid.E, E_STAGGER), (grid.B, B_STAGGER)):
        vals = []
        for c in range(3):
            idx, wts = [], []
            for ax in range(3):
                if grid.active(ax):
                    nodes, w = _stencil(pos[ax], stag[c][ax])
                    idx.append(np.mod(nodes, grid.n[ax]))
                    wts.append(w)
                else:
                    idx.append(np.floor(pos[ax]).astype(np.int64)[None, :] % grid.n[ax])
                    wts.append(np.ones((1, pos.shape[1])))
            acc = np.zeros(pos.shape[1])
            arr = comps[c]
            for a in range(idx[0].shape[0]):
                for b in range(idx[1].shape[0]):
                    for cc in range(idx[2].shape[0]):
                        acc += (arr[idx[2][cc], idx[1][b], idx[0][a]]
                                * wts[0][a] * wts[1][b] * wts[2][cc])
            vals.append(acc)
        out.append(np.stack(vals))
    return out[0], out[1]


def lab_positions(grid, pos, y_slice):
    """Lab coordinates of particles; on (x, z) grids y is the pulse's slice."""
    X = grid.x_min[0] + pos[0] * grid.dx[0]
    Z = grid.x_min[2] + pos[2] * grid.dx[2]
    if grid.dim == 3:
        Y = grid.x_min[1] + pos[1] * grid.dx[1]
    else:
        Y = np.full_like(X, y_slice)
    return X, Y, Z


# ----------------------------------------------------------------------------
# Push
# ----------------------------------------------------------------------------

def boris(u, E, B, q_over_m, dt):
    """Relativistic Boris rotation: u^{n-1/2} -> u^{n+1/2} in fields (E, B).

    Half electric kick, magnetic rotation through t = kappa B / gamma^- with
    s = 2 t / (1 + |t|^2), half electric kick, with kappa = (q/m) dt / 2.
    """
    kappa = 0.5 * q_over_m * dt
    um = u + kappa * E
    gm = np.sqrt(1.0 + np.sum(um * um, axis=0))
    t = kappa * B / gm
    s = 2.0 * t / (1.0 + np.sum(t * t, axis=0))
    uprime = um + np.cross(um, t, axis=0)
    up = um + np.cross(uprime, s, axis=0)
    return up + kappa * E


def gamma_of(u):
    return np.sqrt(1.0 + np.sum(u * u, axis=0))


# ----------------------------------------------------------------------------
# Charge-conserving deposition (Esirkepov, quadratic shape)
# ----------------------------------------------------------------------------

def esirkepov(grid, q, w, pos0, pos1, u_half):
    """Add the current of particles moving pos0 -> pos1 during one step to grid.J.

    The current is built so that the discrete continuity equation
    (rho^{n+1} - rho^n)/dt + div_h J = 0 holds exactly with rho deposited by
    the same quadratic shape at the nodes.  Per active axis a:
        W_a = DS_a * (weighted sum of the other axes' old shape and change),
        J_a(i + 1/2) - J_a(i - 1/2) = -q w (dx_a / dt) W_a(i);
    a 2-D grid's out-of-plane current is q w v_y times the time-averaged
    shape product.  Positions pos0/pos1 are unwrapped cell coordinates.
    """
    dt = grid.dt
    N = pos0.shape[1]
    win = 6
    base, S0, DS = [], [], []
    for ax in range(3):
        if grid.active(ax):
            b = np.floor(pos0[ax]).astype(np.int64) - 2
            nodes = b[:, None] + np.arange(win)[None, :]
            s0 = tsc(pos0[ax][:, None] - nodes)
            s1 = tsc(pos1[ax][:, None] - nodes)
            base.append(b)
            S0.append(s0)
            DS.append(s1 - s0)
        else:
            base.append(np.floor(pos0[ax]).astype(np.int64))
            S0.append(np.ones((N, 1)))
            DS.append(np.zeros((N, 1)))
    qw = q * w
    sx0, sy0, sz0 = S0
    dsx, dsy, dsz = DS
    # Broadcast to (N, wx, wy, wz)
    X0 = sx0[:, :, None, None]; DX = dsx[:, :, None, None]
    Y0 = sy0[:, None, :, None]; DY = dsy[:, None, :, None]
    Z0 = sz0[:, None, None, :]; DZ = dsz[:, None, None, :]
    Wx = DX * (Y0 * Z0 + 0.5 * DY * Z0 + 0.5 * Y0 * DZ + DY * DZ / 3.0)
    Wy = DY * (X0 * Z0 + 0.5 * DX * Z0 + 0.5 * X0 * DZ + DX * DZ / 3.0)
    Wz = DZ * (X0 * Y0 + 0.5 * DX * Y0 + 0.5 * X0 * DY + DX * DY / 3.0)
    gam = gamma_of(u_half)
    Jcomp = []
    for ax, W in ((0, Wx), (1, Wy), (2, Wz)):
        if grid.active(ax):
            # cumulative sum along the axis gives J at the half nodes above each node
            cum = np.cumsum(W, axis=1 + ax)
            Jcomp.append(-(qw * grid.dx[ax] / dt)[:, None, None, None] * cum)
        else:
            v = u_half[ax] / gam
            shape_avg = (X0 * Y0 * Z0 + 0.5 * DX * Z0 * Y0 + 0.5 * X0 * DZ * Y0
                         + DX * DZ * Y0 / 3.0)
            Jcomp.append((qw * v)[:, None, None, None] * shape_avg)
    ii = (base[0][:, None, None, None] + np.arange(Jcomp[0].shape[1])[None, :, None, None])
    jj = (base[1][:, None, None, None] + np.arange(Jcomp[0].shape[2])[None, None, :, None])
    kk = (base[2][:, None, None, None] + np.arange(Jcomp[0].shape[3])[None, None, None, :])
    ii = np.mod(np.broadcast_to(ii, Jcomp[0].shape), grid.n[0])
    jj = np.mod(np.broadcast_to(jj, Jcomp[0].shape), grid.n[1])
    kk = np.mod(np.broadcast_to(kk, Jcomp[0].shape), grid.n[2])
    for c in range(3):
        np.add.at(grid.J[c], (kk.ravel(), jj.ravel(), ii.ravel()), Jcomp[c].ravel())


# ----------------------------------------------------------------------------
# Yee update of E2, B2
# ----------------------------------------------------------------------------

def _dplus(F, grid, ax):
    if not grid.active(ax):
        return 0.0
    return (np.roll(F, -1, axis=_AXIS_OF[ax]) - F) / grid.dx[ax]


def _dminus(F, grid, ax):
    if not grid.active(ax):
        return 0.0
    return (F - np.roll(F, 1, axis=_AXIS_OF[ax])) / grid.dx[ax]


def _b_half(grid):
    """B <- B - (dt/2) curl E  (first and third lines of Eqs. (7)-(9))."""
    Ex, Ey, Ez = grid.E
    h = 0.5 * grid.dt
    cx = _dplus(Ez, grid, 1) - _dplus(Ey, grid, 2)
    cy = _dplus(Ex, grid, 2) - _dplus(Ez, grid, 0)
    cz = _dplus(Ey, grid, 0) - _dplus(Ex, grid, 1)
    grid.B[0] = grid.B[0] - h * cx
    grid.B[1] = grid.B[1] - h * cy
    grid.B[2] = grid.B[2] - h * cz
    if grid.open_x:
        # the transverse B nodes at nx - 1/2 lie outside the open domain
        grid.B[1][..., -1] = 0.0
        grid.B[2][..., -1] = 0.0


def _e_full(grid, source=None):
    """E <- E + dt (curl B - J)  (second line of Eqs. (7)-(9), with Eq. (2)).

    Open x ends: the transverse E at the boundary nodes follows App. B.  At
    x_min Ampere's law with the B node half a cell outside, together with
    the incoming-wave condition averaged over the step (E_y + B_z = 2 S_y,
    E_z - B_y = 2 S_z), is solved for the new boundary E; at x_max the same
    with no incoming wave (E_y - B_z = 0, E_z + B_y = 0).  With
    r = dx/(c dt) this gives
        x_min: (1 + r) E_y' = 4 S_y - 2 B_z(1/2) + (r - 1) E_y
               (1 + r) E_z' = 4 S_z + 2 B_y(1/2) + (r - 1) E_z
        x_max: (1 + r) E_y' = 2 B_z(nx - 3/2) + (r - 1) E_y
               (1 + r) E_z' = -2 B_y(nx - 3/2) + (r - 1) E_z
    (B at the half step, as in the bulk update; J is not applied at the
    boundary nodes).  ``source`` is (S_y, S_z) per row of x nodes ((z, y)
    order) at t^{n+1/2}, or None."""
    Bx, By, Bz = grid.B
    dt = grid.dt
    if grid.open_x:
        old_y = grid.E[1][..., [0, -1]].copy()
        old_z = grid.E[2][..., [0, -1]].copy()
    cx = _dminus(Bz, grid, 1) - _dminus(By, grid, 2)
    cy = _dminus(Bx, grid, 2) - _dminus(Bz, grid, 0)
    cz = _dminus(By, grid, 0) - _dminus(Bx, grid, 1)
    grid.E[0] = grid.E[0] + dt * (cx - grid.J[0])
    grid.E[1] = grid.E[1] + dt * (cy - grid.J[1])
    grid.E[2] = grid.E[2] + dt * (cz - grid.J[2])
    if grid.open_x:
        r = grid.dx[0] / dt
        shape = grid.E[1][..., 0].shape
        sy, sz = (0.0, 0.0) if source is None else (np.reshape(source[0], shape), np.reshape(source[1], shape))
        grid.E[1][..., 0] = (4.0 * sy - 2.0 * Bz[..., 0] + (r - 1.0) * old_y[..., 0]) / (1.0 + r)
        grid.E[2][..., 0] = (4.0 * sz + 2.0 * By[..., 0] + (r - 1.0) * old_z[..., 0]) / (1.0 + r)
        grid.E[1][..., -1] = (2.0 * Bz[..., -2] + (r - 1.0) * old_y[..., 1]) / (1.0 + r)
        grid.E[2][..., -1] = (-2.0 * By[..., -2] + (r - 1.0) * old_z[..., 1]) / (1.0 + r)


def yee_step(grid, source=None):
    """One split Yee step of the internal fields only (Eq. (4)); ``source``
    drives the incoming-wave boundary of an open-x grid."""
    _b_half(grid)
    _e_full(grid, source)
    _b_half(grid)


def incoming_wave_s0(dx, dt):
    """S0/E0 of the incoming-wave boundary (App. B, the exact first form):
    the source amplitude that launches a plane wave of amplitude E0 into the
    Yee bulk, k being the vacuum Yee wavenumber of omega = 1 (Eq. (10)).
    dx, dt internal units (c = omega = 1)."""
    k = _units.dispersion(_units.DISP_EXACT, dx, dt)[3]
    r = dx / dt
    h = 0.5 * dt
    return 0.5 * (math.cos(h) + r * math.sin(h) * math.cos(0.5 * k * dx) / math.sin(0.5 * k * dx))


def boundary_source(grid, pulse, t):
    """(S_y, S_z) per row at time t for a pulse launched through the x_min
    boundary: S0/E0 times the pulse's transverse E at (x_min, row) (App. B;
    the source carries the pulse's own envelope and phase at the boundary)."""
    nz, ny = grid.n[2], grid.n[1]
    kk, jj = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
    X = np.full(kk.shape, grid.x_min[0])
    Y = grid.x_min[1] + jj * grid.dx[1] if grid.dim == 3 else np.full(kk.shape, pulse.q_slice)
    Z = grid.x_min[2] + kk * grid.dx[2]
    E1 = _pulses.analytic_fields(pulse, t, X, Y, Z)[0]
    s0 = incoming_wave_s0(grid.dx[0], grid.dt)
    return s0 * np.asarray(E1[1], dtype=float), s0 * np.asarray(E1[2], dtype=float)


# ----------------------------------------------------------------------------
# One full step
# ----------------------------------------------------------------------------

def sample_pulse(grid, pulse):
    """E1, B1 sampled on the grid at time grid.t: each component at its own
    staggered node (the literal loop of Fig. 1).  On (x, z) grids the lab y
    of every node is the pulse's slice.  Returns (E1[3], B1[3]) shaped like
    grid.E."""
    nx, ny, nz = grid.n
    ii = np.arange(nx)[None, None, :]
    jj = np.arange(ny)[None, :, None]
    kk = np.arange(nz)[:, None, None]
    shape = (nz, ny, nx)
    out = []
    for stag, which in ((E_STAGGER, 0), (B_STAGGER, 1)):
        comps = []
        for c in range(3):
            X = np.broadcast_to(grid.x_min[0] + (ii + stag[c][0]) * grid.dx[0], shape)
            Z = np.broadcast_to(grid.x_min[2] + (kk + (stag[c][2] if grid.active(2) else 0.0)) * grid.dx[2], shape)
            if grid.dim == 3:
                Y = np.broadcast_to(grid.x_min[1] + (jj + stag[c][1]) * grid.dx[1], shape)
            else:
                Y = np.full(shape, pulse.q_slice)
            F = _pulses.analytic_fields(pulse, grid.t, X, Y, Z)[which]
            comps.append(np.array(F[c], dtype=float))
        out.append(comps)
    return out[0], out[1]


def sample_current(grid, pulse, t):
    """Analytic current J1 (Sec. IV) on the grid at time t, each component at
    the node of the matching E component (where the Yee update uses J).
    Returns J1[3] shaped like grid.J."""
    nx, ny, nz = grid.n
    ii = np.arange(nx)[None, None, :]
    jj = np.arange(ny)[None, :, None]
    kk = np.arange(nz)[:, None, None]
    shape = (nz, ny, nx)
    out = []
    for c in range(3):
        stag = E_STAGGER[c]
        X = np.broadcast_to(grid.x_min[0] + (ii + stag[0]) * grid.dx[0], shape)
        Z = np.broadcast_to(grid.x_min[2] + (kk + (stag[2] if grid.active(2) else 0.0)) * grid.dx[2], shape)
        if grid.dim == 3:
            Y = np.broadcast_to(grid.x_min[1] + (jj + stag[1]) * grid.dx[1], shape)
        else:
            Y = np.full(shape, pulse.q_slice)
        out.append(np.array(_pulses.analytic_current(pulse, t, X, Y, Z)[c], dtype=float))
    return out


def push_species(grid, sp, pulse, n_steps_done=None, pulse_on_grid=False, with_fields=False):
    """Field evaluation and Boris push of one species at time grid.t.

    Returns u^{n+1/2} (and the total E, B at the particles with
    ``with_fields``); positions are not changed.
    """
    if pulse is not None and pulse_on_grid:
        E1g, B1g = sample_pulse(grid, pulse)
        saved = grid.E, grid.B
        grid.E = [a + b for a, b in zip(saved[0], E1g)]
        grid.B = [a + b for a, b in zip(saved[1], B1g)]
        try:
            E, B = gather(grid, sp.pos)
        finally:
            grid.E, grid.B = saved
        u1 = boris(sp.u, E, B, sp.q / sp.m, grid.dt)
        return (u1, E, B) if with_fields else u1
    E2, B2 = gather(grid, sp.pos)
    if pulse is not None:
        X, Y, Z = lab_positions(grid, sp.pos, pulse.q_slice)
        E1, B1 = _pulses.analytic_fields(pulse, grid.t, X, Y, Z)
        E = E1 + E2
        B = B1 + B2
    else:
        E, B = E2, B2
    u1 = boris(sp.u, E, B, sp.q / sp.m, grid.dt)
    return (u1, E, B) if with_fields else u1


def move(grid, pos, u_half):
    """x^{n+1} = x^n + dt u^{n+1/2}/gamma^{n+1/2} (cell units, unwrapped)."""
    gam = gamma_of(u_half)
    new = pos.copy()
    for ax in range(3):
        if grid.active(ax):
            new[ax] = pos[ax] + grid.dt * u_half[ax] / gam / grid.dx[ax]
    return new


def wrap(grid, pos):
    out = pos.copy()
    for ax in range(3):
        if grid.active(ax):
            out[ax] = np.mod(pos[ax], grid.n[ax])
    return out


def step(grid, species, pulse, field_update=True, pulse_on_grid=False, launch=False):
    """One step of the loop of Fig. 1.

    ``launch`` (an open-x grid and a plane pulse): the traditional run the
    paper compares with.  The pulse is not evaluated analytically anywhere;
    it enters through the incoming-wave boundary at x_min, and the particles
    feel E2, B2 alone.

    For each species: E = E1 + E2, B = B1 + B2 at x^n, t^n (E1, B1 at the
    particle, or sampled on the grid with ``pulse_on_grid``); Boris push
    (plus the emission proxy of the step for species that carry one); move;
    deposit J^{n+1/2}.  With an analytic current (Sec. IV) J1 at
    t^{n+1/2} is subtracted: E2, B2 are driven by J - J1.  Then the Yee update
    of E2, B2.  J holds the Yee source (J, or J - J1) afterwards.  Returns per-species (pos_unwrapped_new,)
    for diagnostics.
    """
    if launch and not (grid.open_x and pulse is not None and pulse.kind == "plane" and not pulse.current):
        raise ValueError("launching through the boundary needs an open-x grid and a plane pulse")
    for c in range(3):
        grid.J[c][...] = 0.0
    moved = []
    for sp in species:
        u_half, E, B = push_species(grid, sp, None if launch else pulse, pulse_on_grid=pulse_on_grid,
                                    with_fields=True)
        if sp.proxy is not None:
            sp.proxy = sp.proxy + emission_proxy(sp.u, u_half, E, B, grid.dt)
        new = move(grid, sp.pos, u_half)
        disp = np.abs(new - sp.pos)
        if np.any(disp >= 1.0):
            raise ValueError("a particle moved a full cell or more in one step")
        esirkepov(grid, sp.q, sp.w, sp.pos, new, u_half)
        sp.u = u_half
        moved.append(new)
        sp.pos = wrap(grid, new)
    if pulse is not None and pulse.current:
        J1 = sample_current(grid, pulse, grid.t + 0.5 * grid.dt)
        for c in range(3):
            grid.J[c] -= J1[c]
    if field_update:
        yee_step(grid, boundary_source(grid, pulse, grid.t + 0.5 * grid.dt) if launch else None)
    grid.t += grid.dt
    return moved


def shift_window(grid, species, injected, direction=1):
    """Moving window (Sec. III.C: a window that follows the pulse, e.g. the
    intensity peak of a flying focus at v_f of either sign): move it one
    cell along +x (direction 1) or -x (direction -1).

    Lab positions are kept.  Along +x: x_min[0] grows by dx, E2/B2 move down
    one index along x and the new last column is empty; particles move down
    one cell index and those in the first column fall behind the window.
    Along -x: x_min[0] falls by dx, E2/B2 move up one index and the new first
    column is empty; particles move up one cell index and those in the last
    column fall out.  Particles that leave are removed (their ids join the
    free ids).  ``injected`` holds, per species, None or (pos (3, k) in cell
    units of the new window, u (3, k), w (k)): the particles of the entering
    column, which take the k smallest free ids."""
    if direction not in (1, -1):
        raise ValueError("direction must be +1 or -1")
    nx = grid.n[0]
    grid.x_min = (grid.x_min[0] + direction * grid.dx[0],) + tuple(grid.x_min[1:])
    for F in grid.E + grid.B:
        if direction == 1:
            F[..., :-1] = F[..., 1:].copy()
            F[..., -1] = 0.0
        else:
            F[..., 1:] = F[..., :-1].copy()
            F[..., 0] = 0.0
    for sp, inj in zip(species, injected):
        keep = sp.pos[0] >= 1.0 if direction == 1 else sp.pos[0] < nx - 1.0
        if sp.ids is not None:
            sp.free = np.sort(np.concatenate([sp.free, sp.ids[~keep]]))
            sp.ids = sp.ids[keep]
        sp.pos = sp.pos[:, keep]
        sp.pos[0] -= direction
        sp.u = sp.u[:, keep]
        sp.w = sp.w[keep]
        if sp.proxy is not None:
            sp.proxy = sp.proxy[keep]
        if inj is None:
            continue
        pos, u, w = (np.asarray(a, dtype=float) for a in inj)
        k = w.shape[0]
        if sp.ids is not None:
            if k > sp.free.shape[0]:
                raise ValueError("not enough free ids for the injected particles")
            sp.ids = np.concatenate([sp.ids, sp.free[:k]])
            sp.free = sp.free[k:]
        sp.pos = np.concatenate([sp.pos, pos], axis=1)
        sp.u = np.concatenate([sp.u, u], axis=1)
        sp.w = np.concatenate([sp.w, w])
        if sp.proxy is not None:
            sp.proxy = np.concatenate([sp.proxy, np.zeros(k)])


def window_due(x_min, dx, t, beta, x_ref, t_ref):
    """Shift due for a window whose x_min should be x_ref + beta (t - t_ref)
    (Sec. III.C, a window moving with the flying focus at v_f = beta c):
    +1 when that position lies half a cell or more ahead, -1 when it lies
    more than half a cell behind, else 0 (the half-open interval keeps a tie
    from shifting back and forth)."""
    d = (x_ref + beta * (t - t_ref) - x_min) / dx
    return 1 if d >= 0.5 else (-1 if d < -0.5 else 0)


def emission_proxy(u0, u1, E, B, dt):
    """Radiated-power proxy of one step (Lienard form with the 2 r_e/3 factor dropped):
    gamma^2 [ |E + beta x B|^2 - (beta . E)^2 ] dt, with u_bar = (u0 + u1)/2."""
    ub = 0.5 * (u0 + u1)
    g = gamma_of(ub)
    beta = ub / g
    F = E + np.cross(beta, B, axis=0)
    return g ** 2 * (np.sum(F * F, axis=0) - np.sum(beta * E, axis=0) ** 2) * dt


def gridless_step(t, dt, X, u, q_over_m, pulse, with_proxy=False):
    """Test-particle step with no grid: analytic fields only, FP64 lab positions.

    X has shape (3, N) (internal units).  Returns (X^{n+1}, u^{n+1/2}) and, with
    ``with_proxy``, the step's emission-proxy increment.
    """
    E, B = _pulses.analytic_fields(pulse, t, X[0], X[1], X[2])
    u_new = boris(u, E, B, q_over_m, dt)
    gam = gamma_of(u_new)
    X_new = X + dt * u_new / gam
    if with_proxy:
        return X_new, u_new, emission_proxy(u, u_new, E, B, dt)
    return X_new, u_new
