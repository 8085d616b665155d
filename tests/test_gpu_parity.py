"""HIP path vs FP64 oracle, element by element on the same seeded inputs.

Per-step tolerances (reading of the stated accuracy targets):
* momenta: |du| <= tol * max(|u^{n+1/2}|, |u^{n-1/2}|, |q/m| dt |E_tot|), tol = 1e-6 (FP32
  path) and 1e-12 (FP64 path);
* positions: |dx| <= 1e-6 cell (FP32) / 1e-12 (FP64);
* current and fields: |dJ| <= tol * max|J|, |dF| <= tol * max|F| (atomic summation
  order differs, so the FP32 bound is set by accumulation: 2e-6).
All runs go through the C ABI (libapt.so) via the ctypes binding.
"""
import math

import numpy as np
import pytest

from oracle import pic, pulses, units
from tests import cases

pytestmark = pytest.mark.gpu

L = units.LAMBDA


def _run_one_step(case, precision, tile=(0, 0, 0), pulse_on_grid=False):
    sim = cases.sim_from_case(case, precision=precision, tile=tile, pulse_on_grid=pulse_on_grid)
    try:
        g, sps, P = cases.oracle_state(case)
        u_old = [sp.u.copy() for sp in sps]
        fscale = cases.force_scale(g, sps, P)
        pic.step(g, sps, P, pulse_on_grid=pulse_on_grid)
        sim.step(1)
        out = [sim.state(i) for i in range(len(sps))]
        E, B, J = sim.field_views()
        gf = [t.double().cpu().numpy() for t in E + B + J]
        d, st = sim.diag()
        return g, sps, u_old, fscale, out, gf, d
    finally:
        sim.close()


@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
@pytest.mark.parametrize("pulse", ["cfg2", "cfg1"])
@pytest.mark.parametrize("tile", [(0, 0, 0), (16, 1, 8), (32, 1, 16)])
def test_one_step_2d_parity(precision, tol, pulse, tile):
    """One full step (gather + LG/Gaussian field + Boris + move + Esirkepov + Yee) on a
    70x40 grid (several tiles: the default 32x8, 16x8 or 32x16 -- compiled-in shapes and
    one read at run time -- plus ragged tails), electrons and
    protons."""
    if pulse == "cfg1":
        case = cases.make_case(n=(70, 1, 40), x_min=(0.0, 0.0, 0.0), t0_steps=150, pulse="cfg1",
                               u_scale=50.0, seed=3)
    else:
        case = cases.make_case(seed=2, u_scale=20.0)
    g, sps, u_old, fscale, out, gf, d = _run_one_step(case, precision, tile)
    n = case["n"]
    for sp, u0, fs, st in zip(sps, u_old, fscale, out):
        scale = np.maximum(np.maximum(np.linalg.norm(sp.u, axis=0), np.linalg.norm(u0, axis=0)), fs)
        du = np.linalg.norm(st["u"].astype(float) - sp.u, axis=0)
        rel = du / scale
        assert rel.max() <= tol, (rel.max(), np.argmax(rel))
        pos = cases.gpu_positions(case, st)
        for ax in (0, 2):
            dpos = cases.periodic_diff(pos[ax], sp.pos[ax], n[ax])
            assert np.abs(dpos).max() <= (1e-6 if precision == "f32" else 1e-12), (ax, np.abs(dpos).max())
    jmax = max(np.abs(c).max() for c in g.J)
    assert jmax > 0
    ftol = 2e-6 if precision == "f32" else 1e-12
    for k in range(3):
        assert np.abs(gf[6 + k] - g.J[k]).max() <= ftol * jmax, ("J", k)
    for k in range(3):
        fmax = max(np.abs(c).max() for c in g.E + g.B)
        assert np.abs(gf[k] - g.E[k]).max() <= ftol * fmax, ("E", k)
        assert np.abs(gf[3 + k] - g.B[k]).max() <= ftol * fmax, ("B", k)
    assert d.n_nonfinite == 0 and d.n_fast == 0


def test_multistep_fp64_with_sort_and_drift():
    """FP64 path: 12 steps with re-sorting every 4 steps (particles drift across tiles
    between sorts and use the global path) stay at round-off from the oracle."""
    case = cases.make_case(n=(40, 1, 36), x_min=(0.0, 0.0, 0.0), t0_steps=150, pulse="cfg1",
                           u_scale=400.0, seed=5, ppc=3, species=("e",))
    from paper_2307_04843_amd.sim import Simulation  # noqa: F401
    sim = cases.sim_from_case(case, precision="f64", tile=(8, 1, 8), sort_every=4)
    try:
        g, sps, P = cases.oracle_state(case)
        for _ in range(12):
            pic.step(g, sps, P)
        sim.step(12)
        st = sim.state(0)
        sp = sps[0]
        du = np.abs(st["u"] - sp.u).max() / max(1.0, np.abs(sp.u).max())
        assert du < 1e-10
        pos = cases.gpu_positions(case, st)
        for ax in (0, 2):
            assert np.abs(cases.periodic_diff(pos[ax], sp.pos[ax], case["n"][ax])).max() < 1e-10
        E, B, J = sim.field_views()
        fmax = max(np.abs(c).max() for c in g.E + g.B)
        for k in range(3):
            assert np.abs(E[k].cpu().numpy() - g.E[k]).max() < 1e-10 * fmax
    finally:
        sim.close()


@pytest.mark.parametrize("tile", [(0, 0, 0), (8, 8, 4)])
def test_multistep_fp64_3d_fused_resort(tile):
    """FP64 3-D run of 15 steps in ap_step calls of 1, 4, 1, 5 and 4 steps, fast
    electrons and protons crossing tile faces every step.  After the first full
    sort, each push writes the particles' ranks in their new tiles and the next
    push reads through the permutation built from them into the other buffer;
    each call ends with the state back in the caller's arrays.  Every particle
    (by id) and the fields stay at round-off from the oracle."""
    dxl = 0.0625
    n = (20, 18, 14)
    dt = units.default_dt(dxl, 3)
    box = tuple(nn * dxl for nn in n)
    case = cases.make_case(dim=3, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(10.0 / dt), ppc=2,
                           pulse=_gauss_pulse_3d(dxl, dt, box), u_scale=3000.0, seed=23)
    sim = cases.sim_from_case(case, precision="f64", tile=tile)
    try:
        g, sps, P = cases.oracle_state(case)
        for k in (1, 4, 1, 5, 4):
            for _ in range(k):
                pic.step(g, sps, P)
            sim.step(k)
        for i, sp in enumerate(sps):
            st = sim.state(i)
            assert np.array_equal(st["id"], np.arange(sp.u.shape[1]))
            du = np.abs(st["u"] - sp.u).max() / max(1.0, np.abs(sp.u).max())
            assert du < 1e-10, (i, du)
            pos = cases.gpu_positions(case, st)
            for ax in range(3):
                assert np.abs(cases.periodic_diff(pos[ax], sp.pos[ax], n[ax])).max() < 1e-10
            assert np.array_equal(st["w"], sp.w)
        # the particles moved across tiles: not a trivial re-sort
        moved = np.abs(cases.periodic_diff(cases.gpu_positions(case, sim.state(0))[0],
                                           cases.oracle_state(case)[1][0].pos[0], n[0]))
        assert moved.max() > 4.0
        E, B, J = sim.field_views()
        fmax = max(np.abs(c).max() for c in g.E + g.B)
        jmax = max(np.abs(c).max() for c in g.J)
        for k in range(3):
            assert np.abs(E[k].cpu().numpy() - g.E[k]).max() < 1e-10 * fmax
            assert np.abs(B[k].cpu().numpy() - g.B[k]).max() < 1e-10 * fmax
            assert np.abs(J[k].cpu().numpy() - g.J[k]).max() < 1e-10 * jmax
    finally:
        sim.close()


def test_continuity_fp32_on_gpu():
    """The FP32 deposited current satisfies continuity with FP64 charge densities:
    max |(rho1 - rho0)/dt + div J| <= 1e-6 max|J| / dx."""
    from paper_2307_04843_amd import apt
    case = cases.make_case(seed=7, u_scale=20.0)
    sim = cases.sim_from_case(case, precision="f32")
    try:
        sim.step(3, flags=apt.AP_STEP_CONTINUITY)
        d, _ = sim.diag()
        dxi = case["dx"][0] * L
        assert d.j_max > 0
        assert d.continuity_max <= 1e-6 * d.j_max / dxi, (d.continuity_max, d.j_max / dxi)
    finally:
        sim.close()


def test_no_particles_no_internal_field_gpu():
    """Eq. (4) on the GPU: without particles E2 = B2 = J = 0 while the pulse is on."""
    case = cases.make_case(seed=8, field_amp=0.0)
    for sp in case["species"]:
        st = sp["state"]
        for k in ("cell", "w"):
            st[k] = st[k][:0]
        st["off"] = st["off"][:, :0]
        st["u"] = st["u"][:, :0]
    sim = cases.sim_from_case(case)
    try:
        sim.step(5)
        E, B, J = sim.field_views()
        assert all(float(t.abs().max()) == 0.0 for t in E + B + J)
    finally:
        sim.close()


@pytest.mark.parametrize("kind", ["plane", "gauss", "ff"])
@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
def test_gridless_one_step_parity(kind, precision, tol):
    """Gridless test particles: analytic field + Boris + move per particle."""
    from paper_2307_04843_amd import inputs
    from paper_2307_04843_amd.sim import Simulation
    dtl = 0.01
    beam = inputs.beam(4096, 50.0, 0.05, 1.0, 1.0, 0.3, 1.0, seed=3)
    beam["u"][1] = (np.random.default_rng(1).standard_normal(4096) * 2).astype(np.float32)
    prm = dict(a0=3.0, tau=20.0, t_ref=10.0, x_ref=0.0, x_f=0.2, w0=2.0, d_f=3, pol=0,
               dispersion=units.DISP_VACUUM, beta_f=-1.0, x0_ff=0.5, t0_ff=9.0)
    t0 = 9.7
    sim = Simulation(0, dx=(1.0, 1.0, 1.0), x_min=(0.0, 0.0, 0.0), t0=t0, dt=dtl, precision=precision,
                     species=[dict(q=-1.0, m=1.0, state=beam)])
    try:
        sim.set_pulse(kind, **prm)
        sim.step(1)
        st = sim.state(0)
    finally:
        sim.close()
    P = pulses.Pulse(dict(type=kind, **prm))
    X = (beam["icell"].astype(float) + beam["off"].astype(float)) * L
    u0 = beam["u"].astype(float)
    X1, u1 = pic.gridless_step(t0 * L, dtl * L, X, u0, -1.0, P)
    scale = np.maximum(np.maximum(np.linalg.norm(u1, axis=0), np.linalg.norm(u0, axis=0)),
                       np.linalg.norm(u1 - u0, axis=0))
    rel = np.linalg.norm(st["u"] - u1, axis=0) / scale
    assert rel.max() <= tol, rel.max()
    Xg = (st["icell"].astype(float) + st["off"].astype(float)) * L
    assert np.abs(Xg - X1).max() / L <= (1e-6 if precision == "f32" else 1e-12)


def _ff_pulse_3d(dxl, dt, box):
    """Flying-focus pulse for a 3-D replica (lambda units): focus moving at beta_f,
    crossing the replica during the step."""
    return dict(type="ff", a0=2.0, tau=40.0, x_ref=box[0] / 2, t_ref=10.0, x_f=0.0, w0=2.0,
                y_c=box[1] / 2, z_c=box[2] / 2, d_f=3, pol=0, beta_f=-1.0, x0_ff=box[0] / 2,
                t0_ff=10.0, chirp=0.05, dispersion=units.DISP_PAPER2, dx_prop=dxl, dt_prop=dt, dt=dt)


def _gauss_pulse_3d(dxl, dt, box):
    return dict(type="gauss", a0=3.0, tau=20.0, x_ref=box[0] / 2, t_ref=10.0, x_f=box[0] / 2 + 0.3,
                w0=1.0, y_c=box[1] / 2, z_c=box[2] / 2, d_f=3, pol=0, dispersion=units.DISP_PAPER2,
                dx_prop=dxl, dt_prop=dt, dt=dt)


@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
@pytest.mark.parametrize("kind", ["gauss", "ff"])
@pytest.mark.parametrize("tile", [(0, 0, 0), (8, 8, 8)])
def test_one_step_3d_parity(precision, tol, kind, tile):
    """3-D step (27-point gather per component, 4x4x4 Esirkepov window) on a 20x18x14
    grid with 8x4x4 (default) or 8x8x8 tiles (ragged tails on every axis), electrons
    and protons."""
    dxl = 0.0625
    n = (20, 18, 14)
    dt = units.default_dt(dxl, 3)
    box = tuple(nn * dxl for nn in n)
    pp = (_ff_pulse_3d if kind == "ff" else _gauss_pulse_3d)(dxl, dt, box)
    case = cases.make_case(dim=3, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(10.0 / dt),
                           ppc=2, pulse=pp, u_scale=30.0, seed=21)
    g, sps, u_old, fscale, out, gf, d = _run_one_step(case, precision, tile)
    for sp, u0, fs, st in zip(sps, u_old, fscale, out):
        scale = np.maximum(np.maximum(np.linalg.norm(sp.u, axis=0), np.linalg.norm(u0, axis=0)), fs)
        rel = np.linalg.norm(st["u"].astype(float) - sp.u, axis=0) / scale
        assert rel.max() <= tol, (rel.max(), np.argmax(rel))
        pos = cases.gpu_positions(case, st)
        for ax in range(3):
            dpos = cases.periodic_diff(pos[ax], sp.pos[ax], n[ax])
            assert np.abs(dpos).max() <= (1e-6 if precision == "f32" else 1e-12)
    jmax = max(np.abs(c).max() for c in g.J)
    fmax = max(np.abs(c).max() for c in g.E + g.B)
    ftol = 2e-6 if precision == "f32" else 1e-12
    for k in range(3):
        assert np.abs(gf[6 + k] - g.J[k]).max() <= ftol * jmax, ("J", k)
        assert np.abs(gf[k] - g.E[k]).max() <= ftol * fmax, ("E", k)
        assert np.abs(gf[3 + k] - g.B[k]).max() <= ftol * fmax, ("B", k)


def test_continuity_fp32_3d():
    from paper_2307_04843_amd import apt
    dxl = 0.0625
    n = (16, 12, 20)
    dt = units.default_dt(dxl, 3)
    box = tuple(nn * dxl for nn in n)
    case = cases.make_case(dim=3, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(10.0 / dt), ppc=2,
                           pulse=_gauss_pulse_3d(dxl, dt, box), u_scale=30.0, seed=22)
    sim = cases.sim_from_case(case, precision="f32")
    try:
        sim.step(3, flags=apt.AP_STEP_CONTINUITY)
        d, _ = sim.diag()
        assert d.j_max > 0
        assert d.continuity_max <= 1e-6 * d.j_max / (dxl * L)
    finally:
        sim.close()


def _full_run_case():
    from paper_2307_04843_amd import inputs
    dxl = 0.05
    n = (128, 1, 64)
    dt = units.default_dt(dxl, 2)
    st = inputs.plasma(2, n, (dxl,) * 3, (0.0, 0.0, 0.0), 4, inputs.density_uniform(0.01), 1.0, 1.0, seed=1)
    return dict(dim=2, n=n, dx=(dxl,) * 3, x_min=(0.0, 0.0, 0.0), t0=0.0, dt=dt,
                species=[dict(q=-1.0, m=1.0, state=st)],
                fields=[np.zeros((64, 1, 128), np.float32) for _ in range(6)],
                pulse=cases.cfg1_pulse(dxl, dt))


_FULL_RUN = {}


def _oracle_full_run_moments():
    """FP64 oracle moments after the 200-step run (computed once per session)."""
    if "m" not in _FULL_RUN:
        from oracle import diag as odiag
        g, sps, P = cases.oracle_state(_full_run_case())
        for _ in range(200):
            pic.step(g, sps, P)
        _FULL_RUN["m"] = odiag.moments(sps[0])
    return _FULL_RUN["m"]


@pytest.mark.timeout(400)
@pytest.mark.parametrize("precision,tol", [("f64", 1e-9), ("f32", 1e-4)])
def test_full_128x64_gaussian_run_moments(precision, tol):
    """The 128x64-cell 2-D workload end to end: 0.01 n_c electrons at 4 per cell
    (32768), T = 1 eV, paraxial Gaussian a0 = 1, w0 = 5, tau = 10, 200 steps.  Ensemble
    moments after the full run against the FP64 oracle: relative 1e-9 (FP64 path) and
    1e-4 (FP32 path; second moments and <gamma> relative to themselves, first moments
    relative to sqrt(<u^2>))."""
    case = _full_run_case()
    sim = cases.sim_from_case(case, precision=precision)
    try:
        sim.step(200)
        gst = sim.state(0)
        d, _ = sim.diag()
    finally:
        sim.close()
    m = _oracle_full_run_moments()
    ug = gst["u"].astype(float)
    w = gst["w"].astype(float)
    sw = w.sum()
    mean_u = (w * ug).sum(axis=1) / sw
    mean_u2 = (w * ug ** 2).sum(axis=1) / sw
    mean_g = (w * np.sqrt(1 + (ug ** 2).sum(axis=0))).sum() / sw
    ref = np.sqrt(m["mean_u2"].sum())
    assert np.all(np.abs(mean_u - m["mean_u"]) <= tol * ref), (mean_u, m["mean_u"])
    assert np.all(np.abs(mean_u2 - m["mean_u2"]) <= tol * m["mean_u2"]), (mean_u2, m["mean_u2"])
    assert abs(mean_g - m["mean_gamma"]) <= tol * m["mean_gamma"]
    # the GPU's own FP64 diagnostics agree with the host reduction
    assert abs(d.mean_gamma[0] - mean_g) <= 1e-6 * mean_g
    assert m["mean_u2"][2] > 1e-3     # the pulse did drive the plasma


@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
@pytest.mark.parametrize("dim", [2, 3])
def test_one_step_pulse_sampled_on_grid_parity(precision, tol, dim):
    """The paper's literal loop (Fig. 1, AP_SAMPLE_GRID): E1, B1 sampled at the
    staggered Yee nodes and added to E2, B2 before the gather; one full step vs
    the oracle's grid-sampled step.  2-D: the LG pulse of the 4096x1024 run with
    a super-Gaussian envelope on a 70x40 replica; 3-D: the flying focus."""
    if dim == 2:
        case = cases.make_case(seed=12, u_scale=20.0)
        case["pulse"].update(envelope="sgauss", sg_order=4, fwhm=20.0)
    else:
        dxl = 0.0625
        n = (20, 18, 14)
        dt = units.default_dt(dxl, 3)
        box = tuple(nn * dxl for nn in n)
        case = cases.make_case(dim=3, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(10.0 / dt),
                               ppc=2, pulse=_ff_pulse_3d(dxl, dt, box), u_scale=30.0, seed=22)
    g, sps, u_old, fscale, out, gf, d = _run_one_step(case, precision, pulse_on_grid=True)
    n = case["n"]
    for sp, u0, fs, st in zip(sps, u_old, fscale, out):
        scale = np.maximum(np.maximum(np.linalg.norm(sp.u, axis=0), np.linalg.norm(u0, axis=0)), fs)
        rel = np.linalg.norm(st["u"].astype(float) - sp.u, axis=0) / scale
        assert rel.max() <= tol, (rel.max(), np.argmax(rel))
        pos = cases.gpu_positions(case, st)
        for ax in (0, 1, 2) if dim == 3 else (0, 2):
            dpos = cases.periodic_diff(pos[ax], sp.pos[ax], n[ax])
            assert np.abs(dpos).max() <= (1e-6 if precision == "f32" else 1e-12)
    jmax = max(np.abs(c).max() for c in g.J)
    fmax = max(np.abs(c).max() for c in g.E + g.B)
    ftol = 2e-6 if precision == "f32" else 1e-12
    for k in range(3):
        assert np.abs(gf[6 + k] - g.J[k]).max() <= ftol * jmax, ("J", k)
        assert np.abs(gf[k] - g.E[k]).max() <= ftol * fmax, ("E", k)
        assert np.abs(gf[3 + k] - g.B[k]).max() <= ftol * fmax, ("B", k)


def test_many_tiles_sorted_steps_fp64():
    """More tiles than one scan block covers (512 x 160 cells in 4 x 4 tiles:
    5120 tiles, the two-level tile scan), re-sorted every step: two FP64 steps
    vs the oracle, every particle (1 electron + 1 proton per cell)."""
    case = cases.make_case(n=(512, 1, 160), x_min=(0.0, 0.0, 0.0), t0_steps=150, pulse="cfg1", ppc=1,
                           u_scale=20.0, seed=41)
    sim = cases.sim_from_case(case, precision="f64", tile=(4, 1, 4), sort_every=1)
    try:
        g, sps, P = cases.oracle_state(case)
        for _ in range(2):
            pic.step(g, sps, P)
        sim.step(2)
        out = [sim.state(i) for i in range(len(sps))]
        E, B, J = sim.field_views()
        gf = [t.double().cpu().numpy() for t in E + B + J]
    finally:
        sim.close()
    for sp, st in zip(sps, out):
        scale = np.maximum(np.linalg.norm(sp.u, axis=0), 1e-3)
        assert (np.linalg.norm(st["u"].astype(float) - sp.u, axis=0) / scale).max() <= 1e-10
        pos = cases.gpu_positions(case, st)
        for ax in (0, 2):
            assert np.abs(cases.periodic_diff(pos[ax], sp.pos[ax], case["n"][ax])).max() <= 1e-10
    fmax = max(np.abs(c).max() for c in g.E + g.B)
    jmax = max(np.abs(c).max() for c in g.J)
    for k in range(3):
        assert np.abs(gf[k] - g.E[k]).max() <= 1e-10 * fmax
        assert np.abs(gf[3 + k] - g.B[k]).max() <= 1e-10 * fmax
        assert np.abs(gf[6 + k] - g.J[k]).max() <= 1e-10 * jmax
