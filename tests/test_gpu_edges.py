"""Deliberately built edge cases of one step, HIP path vs FP64 oracle.

Each case starts from a seeded replica (2-D: 40 x 24 cells in the LG pulse,
default 16 x 8 tiles with ragged tails; 3-D: 20 x 18 x 14 cells in a
Gaussian pulse, 8 x 4 x 4 tiles) and rewrites the electrons:

* ``offsets``: offsets exactly 0, 0.5 (where the nearest node of the
  staggered gather switches) and 1 - ulp of the working type, on every axis
  in every combination;
* ``faces``: no fields, momenta chosen so that moves end within a few ulps
  of a cell face from either side, or exactly on it (the offset rounding to
  1 or below 0 in the working type must carry into the next cell);
* ``one_cell``: every electron in one cell (same-node atomics in LDS and in
  the flush; that tile holds far more particles than a block covers in one
  pass);
* ``empty``: particles only in the first columns (most tiles empty);
* ``wraps``: particles at both periodic ends of every axis moving across it.

Then the same one-step comparisons as the parity tests: momenta 1e-6 / 1e-12
of their scale, positions 1e-6 / 1e-12 cell, J, E, B node by node 2e-6 /
1e-12 of their maximum, no particle made invalid.
"""
import numpy as np
import pytest

from oracle import pic, units
from tests import cases

pytestmark = pytest.mark.gpu

KINDS = ["offsets", "faces", "one_cell", "empty", "wraps"]


def _gauss_3d(dxl, dt, box):
    return dict(type="gauss", a0=3.0, tau=20.0, x_ref=box[0] / 2, t_ref=10.0, x_f=box[0] / 2 + 0.3,
                w0=1.0, y_c=box[1] / 2, z_c=box[2] / 2, d_f=3, pol=0, dispersion=units.DISP_PAPER2,
                dx_prop=dxl, dt_prop=dt, dt=dt)


def _base(dim, kind):
    nofield = kind == "faces"
    if dim == 2:
        return cases.make_case(n=(40, 1, 24), seed=61, u_scale=20.0, ppc=2,
                               pulse=None if nofield else "cfg2", field_amp=0.0 if nofield else 0.05)
    dxl = 0.0625
    n = (20, 18, 14)
    dt = units.default_dt(dxl, 3)
    box = tuple(nn * dxl for nn in n)
    return cases.make_case(dim=3, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(10.0 / dt), ppc=2,
                           pulse=None if nofield else _gauss_3d(dxl, dt, box), u_scale=30.0, seed=62,
                           field_amp=0.0 if nofield else 0.05)


def _axes(dim):
    return (0, 1, 2) if dim == 3 else (0, 2)


def _edge_case(dim, kind, precision):
    case = _base(dim, kind)
    ft = np.float64 if precision == "f64" else np.float32
    one_minus = np.nextafter(ft(1.0), ft(0.0))
    ulp = ft(1.0) - one_minus
    n = case["n"]
    nx, ny, nz = n[0], (n[1] if dim == 3 else 1), n[2]
    rng = np.random.default_rng(1000 * dim + KINDS.index(kind))
    for sp in case["species"]:
        st = sp["state"]
        for key in ("off", "u", "w"):
            st[key] = st[key].astype(ft)
    e = case["species"][0]["state"]
    N = e["w"].size
    axes = _axes(dim)
    if kind == "offsets":
        vals = np.array([0.0, 0.5, one_minus], dtype=ft)
        for j, ax in enumerate(axes):
            e["off"][ax] = vals[(np.arange(N) // 3 ** j) % 3]
    elif kind == "faces":
        # no field: u is constant and the move is u / gamma * c dt / dx per axis
        cdt = case["dt"] / case["dx"][0]
        k = rng.integers(-4, 5, N)
        for ax in axes:
            up = rng.random(N) < 0.5
            # start 1..8 ulps below the upper face or above the lower one
            steps = rng.integers(1, 9, N).astype(ft)
            e["off"][ax] = np.where(up, one_minus - (steps - 1) * ulp, steps * ulp).astype(ft)
            # moves of (steps + k) ulps towards that face: ends on it, short of it, or just past it
            d = (steps + k) * ulp
            e["u"][ax] = (np.where(up, d, -d) / cdt).astype(ft)
        # a quarter onto the face from 0.75: a move of 0.25 cell needs
        # beta = 0.25 dx / (c dt), u = beta / sqrt(1 - beta^2) (the ulp-sized
        # momenta above leave gamma = 1 in the working type)
        q = N // 4
        beta = 0.25 / cdt
        e["off"][0][:q] = ft(0.75)
        e["u"][0][:q] = ft(beta / np.sqrt(1.0 - beta * beta))
        for ax in axes[1:]:
            e["u"][ax][:q] = ft(0.0)
    elif kind == "one_cell":
        c0 = (nx // 2) + nx * ((ny // 2) + ny * (nz // 2))
        e["cell"] = np.full(N, c0, dtype=np.int32)
        for ax in axes:
            e["off"][ax] = rng.random(N).astype(ft)
    elif kind == "empty":
        for sp in case["species"]:
            st = sp["state"]
            keep = (st["cell"] % nx) < 5
            st["cell"] = st["cell"][keep]
            st["off"], st["u"], st["w"] = st["off"][:, keep], st["u"][:, keep], st["w"][keep]
        e = case["species"][0]["state"]
    elif kind == "wraps":
        # at both ends of every axis, heading out through that end
        side = rng.random(N) < 0.5
        ax = np.array(axes)[rng.integers(0, len(axes), N)]
        idx = [(e["cell"] % nx), (e["cell"] // nx) % ny, e["cell"] // (nx * ny)]
        idx = [i.astype(np.int64) for i in idx]
        ext = (nx, ny, nz)
        for a in axes:
            sel = ax == a
            idx[a][sel] = np.where(side[sel], ext[a] - 1, 0)
            e["off"][a][sel] = np.where(side[sel], ft(0.9), ft(0.1)).astype(ft)
            e["u"][a][sel] = np.where(side[sel], ft(5.0), ft(-5.0)).astype(ft)
        e["cell"] = (idx[0] + nx * (idx[1] + ny * idx[2])).astype(np.int32)
    return case


def _run(case, precision):
    sim = cases.sim_from_case(case, precision=precision)
    try:
        g, sps, P = cases.oracle_state(case)
        u_old = [sp.u.copy() for sp in sps]
        fscale = cases.force_scale(g, sps, P) if P is not None else [np.zeros(sp.u.shape[1]) for sp in sps]
        pic.step(g, sps, P)
        sim.step(1)
        out = [sim.state(i) for i in range(len(sps))]
        E, B, J = sim.field_views()
        gf = [t.double().cpu().numpy() for t in E + B + J]
        d, _ = sim.diag()
        return g, sps, u_old, fscale, out, gf, d
    finally:
        sim.close()


@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("dim", [2, 3])
def test_edge_case_one_step(dim, kind, precision, tol):
    print("edge case", dim, kind, precision, flush=True)
    case = _edge_case(dim, kind, precision)
    g, sps, u_old, fscale, out, gf, d = _run(case, precision)
    n = case["n"]
    ptol = 1e-6 if precision == "f32" else 1e-12
    for sp, u0, fs, st in zip(sps, u_old, fscale, out):
        scale = np.maximum(np.maximum(np.linalg.norm(sp.u, axis=0), np.linalg.norm(u0, axis=0)), fs)
        scale = np.maximum(scale, 1e-30)
        rel = np.linalg.norm(st["u"].astype(float) - sp.u, axis=0) / scale
        assert rel.max() <= tol, (rel.max(), np.argmax(rel))
        pos = cases.gpu_positions(case, st)
        for ax in _axes(case["dim"]):
            dpos = cases.periodic_diff(pos[ax], sp.pos[ax], n[ax])
            assert np.abs(dpos).max() <= ptol, (ax, np.abs(dpos).max())
        # every offset the GPU wrote lies in [0, 1)
        for ax in _axes(case["dim"]):
            assert (st["off"][ax] >= 0).all() and (st["off"][ax] < 1).all()
    assert d.n_nonfinite == 0 and d.n_fast == 0 and d.n_skipped == 0
    jmax = max(np.abs(c).max() for c in g.J)
    assert jmax > 0
    ftol = 2e-6 if precision == "f32" else 1e-12
    for k in range(3):
        assert np.abs(gf[6 + k] - g.J[k]).max() <= ftol * jmax, ("J", k)
    fmax = max(np.abs(c).max() for c in g.E + g.B)
    if fmax > 0:
        for k in range(3):
            assert np.abs(gf[k] - g.E[k]).max() <= ftol * fmax, ("E", k)
            assert np.abs(gf[3 + k] - g.B[k]).max() <= ftol * fmax, ("B", k)
    if kind == "faces":
        # some moves really ended on or across a face: cells changed
        moved = out[0]["cell"] != case["species"][0]["state"]["cell"]   # both in id order
        assert moved.sum() > 0
