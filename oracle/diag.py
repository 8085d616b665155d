"""FP64 diagnostics (oracle): charge density, continuity residual, energies.

These are the quantities the paper inspects (field amplitude, mean electron
energy, total energy: Figs. 2, 3 and 9) plus the discrete continuity
equation that a charge-conserving deposition must satisfy.
"""
import numpy as np

from . import pic


def rho(grid, species):
    """Charge density at the nodes, quadratic shape, periodic."""
    out = np.zeros((grid.n[2], grid.n[1], grid.n[0]))
    for sp in species:
        idx, wts = [], []
        N = sp.pos.shape[1]
        for ax in range(3):
            if grid.active(ax):
                nodes, w = pic._stencil(sp.pos[ax], 0.0)
                idx.append(np.mod(nodes, grid.n[ax]))
                wts.append(w)
            else:
                idx.append(np.floor(sp.pos[ax]).astype(np.int64)[None, :] % grid.n[ax])
                wts.append(np.ones((1, N)))
        for a in range(idx[0].shape[0]):
            for b in range(idx[1].shape[0]):
                for c in range(idx[2].shape[0]):
                    np.add.at(out, (idx[2][c], idx[1][b], idx[0][a]),
                              sp.q * sp.w * wts[0][a] * wts[1][b] * wts[2][c])
    return out


def div_j(grid, J=None):
    """Discrete divergence of J at the nodes (backward differences)."""
    J = grid.J if J is None else J
    out = np.zeros_like(J[0])
    for ax, arr_ax in ((0, 2), (1, 1), (2, 0)):
        if grid.active(ax):
            out += (J[ax] - np.roll(J[ax], 1, axis=arr_ax)) / grid.dx[ax]
    return out


def continuity_residual(grid, rho0, rho1, J=None):
    """(rho^{n+1} - rho^n)/dt + div_h J^{n+1/2}, per node."""
    return (rho1 - rho0) / grid.dt + div_j(grid, J)


def field_energy(grid):
    """Half the sum of E2^2 + B2^2 over cells, times the cell volume: dx dy dz
    in 3-D, dx dz on (x, z) grids (per unit length along y), dx on 1-D rows
    (per unit transverse area of each row, summed over the rows: the rows are
    independent lines, not a slab)."""
    vol = grid.dx[0] * (grid.dx[2] if grid.dim >= 2 else 1.0) * (grid.dx[1] if grid.dim == 3 else 1.0)
    tot = sum(np.sum(c ** 2) for c in grid.E) + sum(np.sum(c ** 2) for c in grid.B)
    return 0.5 * tot * vol


def moments(sp):
    """Weighted particle moments of one species (FP64)."""
    g = pic.gamma_of(sp.u)
    w = sp.w
    sw = np.sum(w)
    # m (gamma - 1) = m |u|^2 / (gamma + 1): the same kinetic energy, without
    # the cancellation of gamma - 1 for slow particles (protons at 1 eV)
    ek = np.sum(sp.u ** 2, axis=0) / (g + 1.0)
    return {
        "sum_w": sw,
        "mean_u": np.sum(w * sp.u, axis=1) / sw,
        "mean_u2": np.sum(w * sp.u ** 2, axis=1) / sw,
        "mean_uperp2": np.sum(w * (sp.u[1] ** 2 + sp.u[2] ** 2)) / sw,
        "mean_gamma": np.sum(w * g) / sw,
        "kinetic": sp.m * np.sum(w * ek),
        "charge": sp.q * sw,
    }
