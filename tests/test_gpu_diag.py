"""FP64 diagnostics of the HIP path (ap_gather_diag) against the oracle.

Every field of ap_diag is compared with the oracle's diagnostics
(``oracle.diag.field_energy``, ``oracle.diag.moments``, the per-particle
proxies) in two ways, on electron + proton runs on (x, z), 3-D and 1-D-row
grids, after several steps inside the pulse:

* on the GPU's own state: the oracle reduces the particles and fields the
  GPU holds (both sides sum the same values in FP64, in different orders):
  1e-12 relative, in FP32 and FP64 runs alike;
* against the oracle's own run from the same inputs: 1e-10 (FP64 path) and
  1e-6 (FP32 path; energies of the fields 1e-5, as E2, B2 agree to 2e-6 of
  their maximum per step).

Then the numeric flags, forced from the host: a NaN momentum and an offset
outside [0, 1) written into particles (AP_E_NUMERIC with the exact counts:
invalid now, pushes skipped since the last call), a momentum whose gamma
overflows the working type (its move dropped and counted), free slots of a
moving window (not counted), and the reset of the step counters at each call.
"""
import math

import numpy as np
import pytest
import torch

from oracle import diag, pic, units
from paper_2307_04843_amd import apt
from tests import cases

pytestmark = pytest.mark.gpu

L = units.LAMBDA
STEPS = 6


def _gauss_pulse_3d(dxl, dt, box):
    return dict(type="gauss", a0=3.0, tau=20.0, x_ref=box[0] / 2, t_ref=10.0, x_f=box[0] / 2 + 0.3,
                w0=1.0, y_c=box[1] / 2, z_c=box[2] / 2, d_f=3, pol=0, dispersion=units.DISP_PAPER2,
                dx_prop=dxl, dt_prop=dt, dt=dt)


def _case(dim):
    if dim == 2:
        return cases.make_case(n=(40, 1, 24), seed=31, u_scale=20.0, ppc=3)
    if dim == 1:
        return cases.make_case(dim=1, n=(64, 1, 4), seed=32, u_scale=20.0, ppc=4, x_min=(48.0, 0.0, 4.4),
                               t0_steps=1343)
    dxl = 0.0625
    n = (16, 12, 10)
    dt = units.default_dt(dxl, 3)
    box = tuple(nn * dxl for nn in n)
    return cases.make_case(dim=3, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(10.0 / dt), ppc=2,
                           pulse=_gauss_pulse_3d(dxl, dt, box), u_scale=30.0, seed=33)


def _oracle_of_gpu_state(case, sim):
    """Oracle grid and species holding the GPU's current fields and particles."""
    g, sps, _ = cases.oracle_state(case)
    E, B, _ = sim.field_views()
    for k in range(3):
        g.E[k][...] = E[k].double().cpu().numpy()
        g.B[k][...] = B[k].double().cpu().numpy()
    out = []
    for i, sp in enumerate(sps):
        st = sim.state(i)
        out.append(pic.Species(sp.q, sp.m, cases.gpu_positions(case, st), st["u"].astype(float),
                               st["w"].astype(float), proxy=st["proxy"]))
    return g, out


def _compare(d, g, sps, tol, tol_fields):
    fe = diag.field_energy(g)
    assert fe > 0
    assert abs(d.field_energy - fe) <= tol_fields * fe, (d.field_energy, fe)
    for i, sp in enumerate(sps):
        m = diag.moments(sp)
        assert abs(d.sum_w[i] - m["sum_w"]) <= tol * m["sum_w"]
        assert abs(d.kinetic[i] - m["kinetic"]) <= tol * m["kinetic"], (i, d.kinetic[i], m["kinetic"])
        assert abs(d.mean_gamma[i] - m["mean_gamma"]) <= tol * m["mean_gamma"]
        u_scale = math.sqrt(sum(m["mean_u2"]))
        for k in range(3):
            assert abs(d.mean_u[i][k] - m["mean_u"][k]) <= tol * u_scale, (i, k)
            assert abs(d.mean_u2[i][k] - m["mean_u2"][k]) <= tol * u_scale ** 2, (i, k)
        pr = float(np.sum(sp.proxy)) if sp.proxy is not None else 0.0
        assert abs(d.proxy_sum[i] - pr) <= tol * abs(pr), (i, d.proxy_sum[i], pr)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3, 1])
def test_diag_matches_oracle(dim, precision):
    case = _case(dim)
    sim = cases.sim_from_case(case, precision=precision, proxy=True)
    try:
        g, sps, P = cases.oracle_state(case, proxy=True)
        for _ in range(STEPS):
            pic.step(g, sps, P)
        sim.step(STEPS)
        d, st = sim.diag()
        assert st == apt.AP_OK
        assert d.step == STEPS
        assert abs(d.t - (case["t0"] + STEPS * case["dt"])) < 1e-12
        assert d.n_nonfinite == 0 and d.n_fast == 0 and d.n_skipped == 0
        # the reductions themselves: the oracle on the GPU's own state
        g_own, sps_own = _oracle_of_gpu_state(case, sim)
        _compare(d, g_own, sps_own, 1e-12, 1e-12)
        # the whole path: the oracle's own run from the same inputs
        if precision == "f64":
            _compare(d, g, sps, 1e-10, 1e-10)
        else:
            _compare(d, g, sps, 1e-6, 1e-5)
    finally:
        sim.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_numeric_flags_forced_from_host(precision):
    """A NaN momentum and an offset of 1.5 written from the host: the next call
    returns AP_E_NUMERIC with n_nonfinite = 2 (invalid now) and no skipped push
    yet; after 3 steps n_skipped = 6 (both skipped every step, left unchanged)
    and the grid stays finite; repaired, the next call is clean.  Then a
    momentum of 1e20 (FP32) or 1e160 (FP64), whose gamma overflows the working
    type: its move is dropped every step (n_fast = steps); in FP32 runs the
    FP64 reductions still hold it as valid, in FP64 runs its gamma overflows
    there too and it counts as invalid."""
    case = cases.make_case(n=(40, 1, 24), seed=34, u_scale=20.0, ppc=2, species=("e",))
    sim = cases.sim_from_case(case, precision=precision)
    try:
        a = sim.arrays[0]
        d, st = sim.diag(allow_numeric=True)
        assert st == apt.AP_OK
        bad_nan, bad_off = 17, 123
        u_keep = a["u"][1][bad_nan].item()
        off_keep = a["off"][0][bad_off].item()
        a["u"][1][bad_nan] = float("nan")
        a["off"][0][bad_off] = 1.5
        torch.cuda.synchronize()
        d, st = sim.diag(allow_numeric=True)
        assert st == apt.AP_E_NUMERIC
        assert d.n_nonfinite == 2 and d.n_skipped == 0 and d.n_fast == 0
        sim.step(3)
        d, st = sim.diag(allow_numeric=True)
        assert st == apt.AP_E_NUMERIC
        assert d.n_nonfinite == 2 and d.n_skipped == 6
        E, B, J = sim.field_views()
        for f in E + B + J:
            assert bool(torch.isfinite(f).all())
        # the skipped particles kept their state (found by id)
        s = sim.state(0)
        assert np.isnan(s["u"][1][bad_nan]) and s["off"][0][bad_off] == np.float32(1.5)
        # repair them (by id: the sort moved them)
        ids = a["id"]
        k_nan = int((ids == bad_nan).nonzero()[0])
        k_off = int((ids == bad_off).nonzero()[0])
        a["u"][1][k_nan] = u_keep
        a["off"][0][k_off] = off_keep
        torch.cuda.synchronize()
        d, st = sim.diag(allow_numeric=True)
        assert st == apt.AP_OK and d.n_nonfinite == 0 and d.n_skipped == 0
        # gamma overflow: the move is dropped and counted, the particle stays valid
        huge = 1e20 if precision == "f32" else 1e160
        k_huge = int((ids == 40).nonzero()[0])
        a["u"][0][k_huge] = huge
        torch.cuda.synchronize()
        before = sim.state(0)
        sim.step(2)
        d, st = sim.diag(allow_numeric=True)
        assert st == apt.AP_E_NUMERIC
        assert d.n_fast == 2 and d.n_skipped == 0
        assert d.n_nonfinite == (0 if precision == "f32" else 1)
        after = sim.state(0)
        assert after["cell"][40] == before["cell"][40]
        assert np.array_equal(after["off"][:, 40], before["off"][:, 40])
        # the counters were reset by the call: nothing happened since
        d, st = sim.diag(allow_numeric=True)
        assert d.n_fast == 0 and d.n_skipped == 0
    finally:
        sim.close()


def test_free_slots_are_not_flagged():
    """Free slots (cell -1, zero state) passed as spare capacity of a moving
    window are neither invalid nor skipped pushes, and add nothing to the sums."""
    from paper_2307_04843_amd import inputs
    case = cases.make_case(n=(40, 1, 24), seed=35, u_scale=20.0, ppc=2, species=("e",))
    full = case["species"][0]["state"]
    n0 = full["w"].shape[0]
    case["species"][0]["state"] = inputs.pad_free(full, 100, n0)
    sim = cases.sim_from_case(case, precision="f64", moving_window=True)
    try:
        sim.step(4)
        d, st = sim.diag()
        assert st == apt.AP_OK
        assert d.n_nonfinite == 0 and d.n_skipped == 0 and d.n_fast == 0
        s = sim.state(0)
        live = s["cell"] >= 0
        assert int(live.sum()) == n0
        assert abs(d.sum_w[0] - float(s["w"][live].astype(float).sum())) <= 1e-12 * d.sum_w[0]
    finally:
        sim.close()
