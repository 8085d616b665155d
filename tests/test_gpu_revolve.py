"""Binomial checkpointing (ap_set_revolve) vs segment checkpoints.

The same recorded run differentiated with both schedules gives the same
gradient: bit for bit in gridless runs (the reverse steps read states that
the same kernels produced from the same inputs), to 1e-12 relative of the
gradient's norm in FP64 gridded runs (a re-advanced step reproduces the
recorded one up to the summation order of the current deposit), in the
frozen-grid and the coupled readings, 2-D and 3-D.  Slot budgets from one
(every step re-advanced from the start) to more than the steps need; the
recording's first descent, the paid recursion and the slotless fallback are
all exercised.  The final state is put back in every case.
"""
import numpy as np
import pytest
import torch

from oracle import units
from paper_2307_04843_amd import apt, inputs
from tests import cases

pytestmark = pytest.mark.gpu


def _gridless(precision, n_steps, segment=None, revolve=None):
    from paper_2307_04843_amd.autograd import GridlessRun
    b = inputs.beam(48, 2000.0, 0.05, 1.0, 1.0, 10.0, 1.0, seed=7)
    pulse = dict(a0=20.0, tau=20.0, t_ref=100.0, x_ref=0.0, x_f=0.0, w0=2.0, np_order=4,
                 dispersion=units.DISP_VACUUM, pol=0)
    return GridlessRun(b, "gauss_np", pulse, ["a0", "w0", "x_f"], n_steps, 0.01, t0=98.0, precision=precision,
                       segment=segment, revolve=revolve)


def _grad(run, values, proxy=True):
    from paper_2307_04843_amd.autograd import APTRun
    p = torch.tensor(values, dtype=torch.float64, requires_grad=True)
    u, pr = APTRun.apply(p, run)
    N = u.shape[1]
    L = (u[1].double() ** 2 + u[2].double() ** 2).sum() / N
    if proxy:
        L = L + 1e-12 * pr.sum() / N
    L.backward()
    return p.grad.numpy().copy(), u.detach().double().cpu().numpy()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_gridless_revolve_equals_segments_bitwise(precision):
    n_steps = 157
    vals = [20.0, 2.0, 0.0]
    run = _gridless(precision, n_steps, segment=12)
    try:
        g_ref, u_ref = _grad(run, vals)
    finally:
        run.close()
    for slots in (1, 2, 5, 13, 200):
        run = _gridless(precision, n_steps, revolve=slots)
        try:
            g, u = _grad(run, vals)
        finally:
            run.close()
        assert np.array_equal(u, u_ref), slots
        assert np.array_equal(g, g_ref), (slots, g, g_ref)


def _case(dim):
    if dim == 2:
        return cases.make_case(n=(24, 1, 16), seed=4, u_scale=10.0, ppc=2)
    dxl = 0.0625
    n = (12, 10, 8)
    dt = units.default_dt(dxl, 3)
    box = tuple(nn * dxl for nn in n)
    pp = dict(type="gauss", a0=3.0, tau=20.0, x_ref=box[0] / 2, t_ref=10.0, x_f=box[0] / 2 + 0.3, w0=1.0,
              y_c=box[1] / 2, z_c=box[2] / 2, d_f=3, pol=1, dispersion=units.DISP_PAPER2, dx_prop=dxl,
              dt_prop=dt, dt=dt)
    return cases.make_case(dim=3, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(10.0 / dt), ppc=2,
                           pulse=pp, u_scale=10.0, seed=23)


def _gridded(case, coupled, n_steps, segment=None, revolve=None):
    from paper_2307_04843_amd.autograd import GriddedRun
    pp = {k: v for k, v in case["pulse"].items() if k not in ("type", "dt")}
    return GriddedRun(case["dim"], case["n"], case["dx"], case["x_min"], case["species"], case["pulse"]["type"],
                      pp, ["a0", "w0", "x_f"], n_steps, t0=case["t0"], dt=case["dt"], precision="f64",
                      fields=case["fields"], segment=segment, sort_every=3, coupled=coupled, revolve=revolve)


def _grad_grid(run, vals):
    """Gradient, final momenta, and whether the reverse sweep put the final
    state (fields, particles) back bit for bit."""
    from paper_2307_04843_amd.autograd import APTRun
    p = torch.tensor(vals, dtype=torch.float64, requires_grad=True)
    u, _ = APTRun.apply(p, run)
    torch.cuda.synchronize()
    E, B, _ = run.sim.field_views()
    before = [t.clone() for t in E + B] + [run.sim.arrays[0]["cell"].clone(), run.sim.arrays[0]["u"][2].clone()]
    N = u.shape[1]
    L = (u[2].double() ** 2).sum() / (2 * N)
    L.backward()
    torch.cuda.synchronize()
    E, B, _ = run.sim.field_views()
    after = [t for t in E + B] + [run.sim.arrays[0]["cell"], run.sim.arrays[0]["u"][2]]
    restored = all(bool(torch.equal(a, b)) for a, b in zip(before, after))
    return p.grad.numpy().copy(), u.detach().double().cpu().numpy(), restored


@pytest.mark.timeout(600)
@pytest.mark.parametrize("coupled", [False, True])
@pytest.mark.parametrize("dim", [2, 3])
def test_gridded_revolve_equals_segments_fp64(dim, coupled):
    print("revolve vs segments, dim", dim, "coupled", coupled, flush=True)
    case = _case(dim)
    n_steps = 13
    vals = [case["pulse"][k] for k in ("a0", "w0", "x_f")]
    run = _gridded(case, coupled, n_steps, segment=4)
    try:
        g_ref, u_ref, restored = _grad_grid(run, vals)
    finally:
        run.close()
    assert restored
    for slots in (1, 3, 6):
        run = _gridded(case, coupled, n_steps, revolve=slots)
        try:
            g, u, restored = _grad_grid(run, vals)
        finally:
            run.close()
        assert restored, slots
        # two forward runs: equal up to the deposit's summation order
        assert np.abs(u - u_ref).max() <= 1e-12 * np.abs(u_ref).max(), slots
        assert np.abs(g - g_ref).max() <= 1e-12 * np.linalg.norm(g_ref), (slots, g, g_ref)


def test_revolve_errors_and_sizes():
    case = _case(2)
    run = _gridded(case, False, 5, segment=2)
    try:
        ctx = run.sim.ctx
        b1 = apt.ap_revolve_bytes(ctx, 1)
        b4 = apt.ap_revolve_bytes(ctx, 4)
        assert b4 > b1 > 0
        # each further slot holds one whole state, whatever the number of steps
        assert (b4 - b1) % 3 == 0
        with pytest.raises(apt.APTError, match="slots"):
            apt.ap_set_revolve(ctx, run.ckpt.data_ptr(), run.ckpt.numel(), 0)
        with pytest.raises(apt.APTError, match="smaller"):
            apt.ap_set_revolve(ctx, run.ckpt.data_ptr(), b4 - 1, 4)
    finally:
        run.close()
