"""Seeded synthetic inputs shared by the HIP path's callers and the oracle.

This module only draws random numbers and lays them out; it holds none of
the method's arithmetic (no fields, no push, no deposition).  Both sides of
every parity test start from the arrays produced here.  All values are
exactly representable in FP32 so that the FP32 and FP64 paths and the oracle
see bit-identical initial states.

Random numbers come from NumPy's Philox-4x32-10 counter-based generator
(Salmon et al. 2011), one stream per (seed, species).  ``plasma_device``
draws the same recipe on the GPU with torch's Philox generator (for inputs of
a billion particles, which the host would take minutes to draw); its streams
differ from NumPy's, so runs started from it are checked against the oracle
on sampled particles, from the GPU's own state.
"""
import math

import numpy as np


def _xp(x):
    """Array module of x: numpy, or torch for torch tensors (device inputs)."""
    if type(x).__module__.split(".")[0] == "torch":
        import torch
        return torch
    return np

ELECTRON_REST_EV = 510998.95
PROTON_MASS = 1836.15267343


def _rng(seed, stream):
    return np.random.Generator(np.random.Philox(key=int(seed) * 1000003 + int(stream)))


def _unit_offsets(rng, n):
    """FP32 offsets uniformly in [0, 1)."""
    v = rng.random(n, dtype=np.float64).astype(np.float32)
    one_minus = np.nextafter(np.float32(1.0), np.float32(0.0))
    return np.minimum(v, one_minus)


def density_uniform(n0):
    return lambda x, y, z: _xp(x).full_like(x, n0)


def density_ramp_x(n0, x_start, length):
    """n = n0 * min(1, (x - x_start)/length) for x >= x_start, else 0 (lambda units)."""
    return lambda x, y, z: n0 * _xp(x).clip((x - x_start) / length, 0.0, 1.0)


def pad_free(state, n_free, first_id):
    """Append n_free free particle slots (cell -1, zero offsets, momentum and
    weight) to a gridded state, with ids first_id, first_id + 1, ...; the
    state's own ids are 0..N-1 (``id`` added when absent)."""
    N = state["w"].shape[0]
    out = dict(state)
    out["id"] = np.concatenate([state.get("id", np.arange(N, dtype=np.int32)).astype(np.int32),
                                np.arange(first_id, first_id + n_free, dtype=np.int32)])
    out["cell"] = np.concatenate([state["cell"], np.full(n_free, -1, np.int32)])
    out["off"] = np.concatenate([state["off"], np.zeros((3, n_free), state["off"].dtype)], axis=1)
    out["u"] = np.concatenate([state["u"], np.zeros((3, n_free), state["u"].dtype)], axis=1)
    out["w"] = np.concatenate([state["w"], np.zeros(n_free, state["w"].dtype)])
    return out


def window_column(dim, n_cells, dx, x_min, ppc, density, temperature_ev, mass, seed, stream=0, column=None):
    """Particles of the column a moving window adds: ``plasma`` on a grid one
    cell wide at window column ``column`` (default the last, n_cells[0] - 1;
    0 for a window moving along -x), i.e. lab x = x_min[0] + column dx[0]
    (x_min is the new window's origin), with cells renumbered into that
    column of the full grid."""
    nx = n_cells[0]
    c = nx - 1 if column is None else int(column)
    col = plasma(dim, (1,) + tuple(n_cells[1:]), dx, (x_min[0] + c * dx[0],) + tuple(x_min[1:]), ppc,
                 density, temperature_ev, mass, seed, stream)
    col["cell"] = (col["cell"].astype(np.int64) * nx + c).astype(np.int32)
    return col


def density_slab_x(n0, x0, x1):
    """n = n0 for x0 <= x < x1, else 0 (lambda units)."""
    return lambda x, y, z: n0 * ((x >= x0) & (x < x1))


def density_gauss_channel(n0, radius, y_axis, z_axis):
    """n = n0 exp(-r_perp^2 / radius^2) about the axis (y_axis, z_axis)."""
    return lambda x, y, z: n0 * _xp(x).exp(-((y - y_axis) ** 2 + (z - z_axis) ** 2) / radius ** 2)


def plasma(dim, n_cells, dx, x_min, ppc, density, temperature_ev, mass, seed,
           stream=0, positions_from=None):
    """Macroparticles filling every cell of a grid, ``ppc`` per cell.

    dim 2 uses axes (x, z); dim 3 uses (x, y, z); dim 1 fills rows of 1-D
    lines along x, row k at z = x_min[2] + k dx[2] (no z offset).  ``dx`` and ``x_min`` are
    per-axis (x, y, z) in lambda units.  Returns a dict of arrays:
        cell  int32 linear cell index (x fastest, then y, then z)
        off   float32 (3, N) offsets in [0, 1) per axis (unused axes zero)
        u     float32 (3, N) momenta gamma*beta, Maxwellian with temperature T
        w     float32 (N,) weights n(x_p)/ppc in units of n_c
    Particles are emitted cell by cell.  ``positions_from`` reuses another
    species' cells and offsets (co-located ions).
    """
    nx, ny, nz = n_cells
    if dim in (1, 2):
        ny = 1
    ncell = nx * ny * nz
    N = ncell * ppc
    rng = _rng(seed, stream)
    if positions_from is None:
        cell = np.repeat(np.arange(ncell, dtype=np.int64), ppc).astype(np.int32)
        off = np.zeros((3, N), dtype=np.float32)
        off[0] = _unit_offsets(rng, N)
        if dim == 3:
            off[1] = _unit_offsets(rng, N)
        if dim >= 2:
            off[2] = _unit_offsets(rng, N)
    else:
        cell = positions_from["cell"].copy()
        off = positions_from["off"].copy()
    sigma = math.sqrt(temperature_ev / (ELECTRON_REST_EV * mass))
    u = (rng.standard_normal((3, N)) * sigma).astype(np.float32)
    i = cell.astype(np.int64) % nx
    j = (cell.astype(np.int64) // nx) % ny
    k = cell.astype(np.int64) // (nx * ny)
    xs = x_min[0] + (i + off[0].astype(np.float64)) * dx[0]
    ys = (x_min[1] + (j + off[1].astype(np.float64)) * dx[1]) if dim == 3 else np.zeros(N)
    zs = x_min[2] + (k + off[2].astype(np.float64)) * dx[2]
    w = (density(xs, ys, zs) / ppc).astype(np.float32)
    return {"cell": cell, "off": off, "u": u, "w": w}


def plasma_device(dim, n_cells, dx, x_min, ppc, density, temperature_ev, mass, seed, stream=0,
                  positions_from=None, device="cuda", chunk=1 << 26):
    """The recipe of ``plasma`` (every cell filled with ``ppc`` particles,
    offsets uniform in [0, 1), Maxwellian momenta, weights n(x_p)/ppc, cell by
    cell) drawn on a torch device with torch's Philox-4x32-10 generator keyed
    by (seed, stream).  Returns device tensors (cell int32, off float32
    (3, N), u float32 (3, N), w float32 (N,)).  ``positions_from`` reuses
    another species' cells and offsets (co-located ions; they are cloned).
    Work proceeds in chunks of ``chunk`` particles to bound the temporaries."""
    import torch
    nx, ny, nz = n_cells
    if dim in (1, 2):
        ny = 1
    ncell = nx * ny * nz
    N = ncell * ppc
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) * 1000003 + int(stream))
    sigma = math.sqrt(temperature_ev / (ELECTRON_REST_EV * mass))
    if positions_from is None:
        cell = torch.arange(ncell, dtype=torch.int32, device=dev).repeat_interleave(ppc)
        off = torch.zeros((3, N), dtype=torch.float32, device=dev)
        axes = (0, 1, 2) if dim == 3 else ((0, 2) if dim == 2 else (0,))
        for a in axes:
            torch.rand(N, generator=gen, dtype=torch.float32, device=dev, out=off[a])
    else:
        cell = positions_from["cell"].clone()
        off = positions_from["off"].clone()
    u = torch.empty((3, N), dtype=torch.float32, device=dev)
    for a in range(3):
        torch.randn(N, generator=gen, dtype=torch.float32, device=dev, out=u[a])
    u *= sigma
    w = torch.empty(N, dtype=torch.float32, device=dev)
    for b in range(0, N, chunk):
        e = min(N, b + chunk)
        c = cell[b:e].to(torch.int64)
        i = c % nx
        j = (c // nx) % ny
        k = c // (nx * ny)
        xs = x_min[0] + (i + off[0, b:e].double()) * dx[0]
        ys = (x_min[1] + (j + off[1, b:e].double()) * dx[1]) if dim == 3 else torch.zeros_like(xs)
        zs = x_min[2] + (k + off[2, b:e].double()) * dx[2]
        w[b:e] = (density(xs, ys, zs) / ppc).float()
    return {"cell": cell, "off": off, "u": u, "w": w}


def beam(n, gamma0, rel_spread, sigma_perp, sigma_long, x_center, vcell, seed,
         stream=0, direction=-1.0):
    """Relativistic electron beam for gridless test-particle runs.

    gamma ~ N(gamma0, (rel_spread*gamma0)^2), moving along x with sign
    ``direction``, no divergence; transverse N(0, sigma_perp^2) per axis and
    longitudinal N(x_center, sigma_long^2) (lambda units).  Positions are
    returned as per-axis int32 virtual cells of size ``vcell`` (lambda) plus
    FP32 offsets, origin at zero.
    """
    rng = _rng(seed, stream)
    g = gamma0 * (1.0 + rel_spread * rng.standard_normal(n))
    g = np.maximum(g, 1.0 + 1e-6)
    ux = direction * np.sqrt(g * g - 1.0)
    pos = np.stack([x_center + sigma_long * rng.standard_normal(n),
                    sigma_perp * rng.standard_normal(n),
                    sigma_perp * rng.standard_normal(n)])
    scaled = pos / vcell
    icell = np.floor(scaled).astype(np.int32)
    off = (scaled - icell).astype(np.float32)
    one_minus = np.nextafter(np.float32(1.0), np.float32(0.0))
    off = np.minimum(off, one_minus)
    u = np.zeros((3, n), dtype=np.float32)
    u[0] = ux.astype(np.float32)
    return {"icell": icell, "off": off, "u": u, "w": np.full(n, 1.0 / n, dtype=np.float32)}
