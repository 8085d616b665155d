"""Rows of independent 1-D grids (the reduced-dimensionality series of Sec.
III.B) on the HIP path vs the oracle.

Each row is a 1D-3V simulation along x at its own lab z (y = the pulse's
slice); the analytic pulse is the full 3-D field there.  Cases: 96 cells x 5
rows at lambda/20 (4 electrons + 4 protons per cell, random E2/B2, u scaled
x20 to cross cells), the LG pulse of the 4096 x 1024 run and a flying focus;
one step (FP32 and FP64, per the tolerances of ``test_gpu_parity``), 20 FP64
steps with re-sorts, continuity in FP32, the grid-sampled loop with an
analytic current, and the frozen-grid adjoint.
"""
import numpy as np
import pytest
import torch

from oracle import grad as ograd
from oracle import pic, units
from tests import cases

pytestmark = pytest.mark.gpu


def _case(pulse="cfg2", seed=51, n=(96, 1, 5), u_scale=20.0, ppc=4):
    # clock at t = 63.8 lambda/c (the 2-D replicas' time): the LG pulse covers the rows
    case = cases.make_case(dim=1, n=n, seed=seed, u_scale=u_scale, ppc=ppc, x_min=(48.0, 0.0, 4.4),
                           t0_steps=1343)
    if pulse == "ff":
        dxl, dt = case["dx"][0], case["dt"]
        case["pulse"] = dict(type="ff", a0=2.0, tau=40.0, x_ref=50.0, t_ref=case["t0"], x_f=0.0, w0=2.0,
                             y_c=0.0, z_c=4.5, d_f=3, pol=1, beta_f=-1.0, x0_ff=50.4, t0_ff=case["t0"],
                             chirp=0.05, dispersion=units.DISP_PAPER2, dx_prop=dxl, dt_prop=dt, dt=dt)
    return case


def _compare(case, g, sps, u_old, fscale, out, gf, tol):
    n = case["n"]
    for sp, u0, fs, st in zip(sps, u_old, fscale, out):
        scale = np.maximum(np.maximum(np.linalg.norm(sp.u, axis=0), np.linalg.norm(u0, axis=0)), fs)
        rel = np.linalg.norm(st["u"].astype(float) - sp.u, axis=0) / scale
        assert rel.max() <= tol, (rel.max(), np.argmax(rel))
        pos = cases.gpu_positions(case, st)
        dpos = cases.periodic_diff(pos[0], sp.pos[0], n[0])
        assert np.abs(dpos).max() <= (1e-6 if tol > 1e-9 else 1e-12)
        assert np.array_equal(pos[2], sp.pos[2])          # rows never change
    jmax = max(np.abs(c).max() for c in g.J)
    fmax = max(np.abs(c).max() for c in g.E + g.B)
    ftol = 2e-6 if tol > 1e-9 else 1e-12
    for k in range(3):
        assert np.abs(gf[6 + k] - g.J[k]).max() <= ftol * jmax, ("J", k)
        assert np.abs(gf[k] - g.E[k]).max() <= ftol * fmax, ("E", k)
        assert np.abs(gf[3 + k] - g.B[k]).max() <= ftol * fmax, ("B", k)


@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
@pytest.mark.parametrize("pulse", ["cfg2", "ff"])
def test_rows1d_one_step_parity(precision, tol, pulse):
    case = _case(pulse)
    print("rows1d one step", pulse, precision, flush=True)
    sim = cases.sim_from_case(case, precision=precision)
    try:
        g, sps, P = cases.oracle_state(case)
        u_old = [sp.u.copy() for sp in sps]
        fscale = cases.force_scale(g, sps, P)
        pic.step(g, sps, P)
        sim.step(1)
        out = [sim.state(i) for i in range(len(sps))]
        E, B, J = sim.field_views()
        gf = [t.double().cpu().numpy() for t in E + B + J]
    finally:
        sim.close()
    _compare(case, g, sps, u_old, fscale, out, gf, tol)


def test_rows1d_multistep_fp64_with_sorts():
    """20 FP64 steps, re-sorted every 3 steps (tiles of 16 cells), vs the oracle."""
    case = _case(seed=52)
    sim = cases.sim_from_case(case, precision="f64", tile=(16, 1, 1), sort_every=3)
    try:
        g, sps, P = cases.oracle_state(case)
        for _ in range(20):
            pic.step(g, sps, P)
        sim.step(20)
        out = [sim.state(i) for i in range(len(sps))]
        E, B, J = sim.field_views()
        gf = [t.double().cpu().numpy() for t in E + B + J]
        d, _ = sim.diag()
    finally:
        sim.close()
    for sp, st in zip(sps, out):
        scale = np.maximum(np.linalg.norm(sp.u, axis=0), 1e-3)
        assert (np.linalg.norm(st["u"].astype(float) - sp.u, axis=0) / scale).max() <= 1e-10
    fmax = max(np.abs(c).max() for c in g.E + g.B)
    for k in range(3):
        assert np.abs(gf[k] - g.E[k]).max() <= 1e-10 * fmax
        assert np.abs(gf[3 + k] - g.B[k]).max() <= 1e-10 * fmax
    assert d.n_nonfinite == 0 and d.n_fast == 0


def test_rows1d_continuity_fp32():
    from paper_2307_04843_amd import apt
    case = _case(seed=53)
    sim = cases.sim_from_case(case, precision="f32")
    try:
        sim.step(5, flags=apt.AP_STEP_CONTINUITY)
        d, _ = sim.diag()
    finally:
        sim.close()
    dxi = case["dx"][0] * units.LAMBDA
    assert d.j_max > 0
    assert d.continuity_max <= 1e-6 * d.j_max / dxi, (d.continuity_max, d.j_max / dxi)


@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
def test_rows1d_grid_sampled_with_analytic_current(precision, tol):
    """The paper's 1-D setting of Sec. IV: a plane pulse in plasma with J1, E1 and
    B1 sampled on the rows' nodes; one step vs the oracle."""
    case = _case(seed=54)
    dxl, dt = case["dx"][0], case["dt"]
    case["pulse"] = dict(type="plane", a0=0.5, tau=30.0, x_ref=50.0, t_ref=case["t0"], pol=1,
                         dispersion=units.DISP_PLASMA, wp2=0.05, dx_prop=dxl, dt_prop=dt, dt=dt,
                         envelope="sgauss", sg_order=2, fwhm=10.0)
    sim = cases.sim_from_case(case, precision=precision, pulse_on_grid=True)
    try:
        g, sps, P = cases.oracle_state(case)
        u_old = [sp.u.copy() for sp in sps]
        fscale = cases.force_scale(g, sps, P)
        pic.step(g, sps, P, pulse_on_grid=True)
        sim.step(1)
        out = [sim.state(i) for i in range(len(sps))]
        E, B, J = sim.field_views()
        gf = [t.double().cpu().numpy() for t in E + B + J]
    finally:
        sim.close()
    _compare(case, g, sps, u_old, fscale, out, gf, tol)


@pytest.mark.timeout(600)
def test_rows1d_frozen_grid_adjoint_fp64():
    """Frozen-grid gradient of <u_z^2>/2 of the electrons wrt (a0, w0, x_f) over
    12 steps of the LG rows (segments of 5), vs the oracle's reference."""
    from paper_2307_04843_amd.autograd import APTRun, GriddedRun
    case = _case(seed=55, n=(48, 1, 4), u_scale=10.0, ppc=2)
    names = ["a0", "w0", "x_f"]
    vals = [case["pulse"][k] for k in names]
    pp = {k: v for k, v in case["pulse"].items() if k not in ("type", "dt")}
    run = GriddedRun(1, case["n"], case["dx"], case["x_min"], case["species"], "lg", pp, names, 12,
                     t0=case["t0"], dt=case["dt"], precision="f64", fields=case["fields"], segment=5,
                     sort_every=3)
    try:
        p = torch.tensor(vals, dtype=torch.float64, requires_grad=True)
        u, _ = APTRun.apply(p, run)
        N = u.shape[1]
        ((u[2].double() ** 2).sum() / (2 * N)).backward()
        gr = p.grad.numpy().copy()
        u_final = u.detach().double().cpu().numpy()
    finally:
        run.close()
    g, sps, _ = cases.oracle_state(case)
    prm = dict(case["pulse"])
    sp0 = pic.Species(sps[0].q, sps[0].m, sps[0].pos, sps[0].u, sps[0].w)
    recs = ograd.record_gridded_run(g, sps, prm, 12)
    wu = np.zeros_like(u_final)
    wu[2] = u_final[2] / u_final.shape[1]
    ref = np.array([ograd.frozen_gradient(prm, nm, g, recs, sp0, wu)[0] for nm in names])
    fine = np.array([ograd.frozen_gradient(prm, nm, g, recs, sp0, wu, rel_h=1e-7)[0] for nm in names])
    assert np.all(np.abs(fine - ref) <= 1e-7 * np.linalg.norm(ref))
    assert np.abs(u_final - sps[0].u).max() <= 1e-9 * np.abs(sps[0].u).max()
    assert np.all(np.abs(gr - ref) <= 1e-6 * np.linalg.norm(ref)), (gr, ref)
