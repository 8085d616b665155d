"""ap_gather_diag_static (reductions in the library's static scratch, no
allocation) against ap_gather_diag (reductions in the context workspace).

Two contexts: a 3-D run of electrons and protons with emission proxies, then
a smaller (x, z) run of electrons only, so the second call on the shared
scratch sees a smaller input than the first and the larger run's sums of its
second species are still in the array.  On the same state both entry points
run the same deterministic reductions, so every field agrees exactly; the
step counters (skipped pushes, continuity maxima) are read and reset by
whichever of the two is called first, in either order.
"""
import math

import pytest
import torch

from oracle import units
from paper_2307_04843_amd import apt
from tests import cases

pytestmark = pytest.mark.gpu

REDUCED = ("sum_w", "mean_u", "mean_u2", "mean_gamma", "kinetic", "proxy_sum")


def _large_case():
    dxl = 0.0625
    n = (16, 12, 10)
    dt = units.default_dt(dxl, 3)
    box = tuple(nn * dxl for nn in n)
    pulse = dict(type="gauss", a0=3.0, tau=20.0, x_ref=box[0] / 2, t_ref=10.0, x_f=box[0] / 2 + 0.3, w0=1.0,
                 y_c=box[1] / 2, z_c=box[2] / 2, d_f=3, pol=0, dispersion=units.DISP_PAPER2, dx_prop=dxl,
                 dt_prop=dt, dt=dt)
    return cases.make_case(dim=3, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(10.0 / dt), ppc=2,
                           pulse=pulse, u_scale=30.0, seed=41)


def _small_case():
    return cases.make_case(n=(40, 1, 24), seed=42, u_scale=20.0, ppc=2, species=("e",))


def _same(a, b):
    return a == b or (math.isnan(a) and math.isnan(b))


def _flat(d):
    out = {}
    for name in REDUCED:
        v = getattr(d, name)
        for i in range(4):
            if name in ("mean_u", "mean_u2"):
                for k in range(3):
                    out["%s[%d][%d]" % (name, i, k)] = v[i][k]
            else:
                out["%s[%d]" % (name, i)] = v[i]
    out["field_energy"] = d.field_energy
    out["t"] = d.t
    out["step"] = d.step
    out["n_nonfinite"] = d.n_nonfinite
    return out


def _assert_reductions_equal(a, b):
    fa, fb = _flat(a), _flat(b)
    bad = {k: (fa[k], fb[k]) for k in fa if not _same(fa[k], fb[k])}
    assert not bad, bad


def _both(sim, static_first, allow_numeric=False):
    """Static and workspace entry points on the same state, in the given order."""
    calls = [apt.ap_gather_diag_static, apt.ap_gather_diag]
    if not static_first:
        calls.reverse()
    first, st1 = calls[0](sim.ctx, allow_numeric=allow_numeric)
    second, st2 = calls[1](sim.ctx, allow_numeric=allow_numeric)
    return (first, st1), (second, st2)


def test_static_diag_matches_workspace_diag():
    big = cases.sim_from_case(_large_case(), precision="f32", proxy=True)
    small = cases.sim_from_case(_small_case(), precision="f64")
    try:
        # 1. the large run: 3-D, two species, continuity maxima accumulated
        big.step(4, apt.AP_STEP_CONTINUITY)
        (ds, st_s), (dw, st_w) = _both(big, static_first=True)
        assert st_s == st_w == apt.AP_OK
        _assert_reductions_equal(ds, dw)
        assert ds.sum_w[1] > 0 and ds.field_energy > 0 and ds.proxy_sum[0] != 0
        assert ds.continuity_max > 0 and ds.j_max > 0
        # the static call read and reset the step counters
        assert dw.continuity_max == 0 and dw.j_max == 0

        # 2. the smaller run, right after: one species on (x, z); one particle
        # made invalid, so its pushes are skipped and counted
        a = small.arrays[0]
        a["u"][1][5] = float("nan")
        torch.cuda.synchronize()
        small.step(3)
        (ds, st_s), (dw, st_w) = _both(small, static_first=True, allow_numeric=True)
        assert st_s == st_w == apt.AP_E_NUMERIC
        _assert_reductions_equal(ds, dw)
        assert ds.n_nonfinite == 1 and ds.n_skipped == 3
        assert dw.n_skipped == 0
        # the large run's second species is still in the scratch: never read back
        assert ds.sum_w[1] == 0 and ds.kinetic[1] == 0 and ds.mean_gamma[1] == 0
        assert ds.sum_w[0] > 0

        # 3. the other order: the workspace call resets, the static one reads zero
        small.step(2)
        (dw, st_w), (ds, st_s) = _both(small, static_first=False, allow_numeric=True)
        assert st_s == st_w == apt.AP_E_NUMERIC
        _assert_reductions_equal(ds, dw)
        assert dw.n_skipped == 2 and ds.n_skipped == 0

        # 4. the large run again, after the smaller one; fields only
        big.step(2)
        ds, st_s = apt.ap_gather_diag_static(big.ctx, apt.AP_DIAG_FIELDS)
        dw, st_w = apt.ap_gather_diag(big.ctx, apt.AP_DIAG_FIELDS)
        assert st_s == st_w == apt.AP_OK
        _assert_reductions_equal(ds, dw)
        assert ds.field_energy > 0 and ds.sum_w[0] == 0
        ds, st_s = apt.ap_gather_diag_static(big.ctx)
        dw, st_w = apt.ap_gather_diag(big.ctx)
        _assert_reductions_equal(ds, dw)
    finally:
        big.close()
        small.close()


def test_static_diag_argument_errors():
    small = cases.sim_from_case(_small_case(), precision="f32")
    try:
        lib = apt.load()
        out = apt.ap_diag()
        assert lib.ap_gather_diag_static(None, apt.AP_DIAG_PARTICLES, apt.C.byref(out)) == apt.AP_E_ARG
        assert lib.ap_gather_diag_static(small.ctx, apt.AP_DIAG_PARTICLES, None) == apt.AP_E_ARG
        assert lib.ap_gather_diag_static(small.ctx, 0x80, apt.C.byref(out)) == apt.AP_E_ARG
    finally:
        small.close()
