"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/apt.h, and validates arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2307_04843_amd import apt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "apt.h")).read()
    return sorted(set(re.findall(r"^(?:ap_status|const char \*)\s*(ap_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = apt.load()
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(apt.EXPORTED)


def _grid(dim=2, n=(64, 1, 32), dx=0.05, prec=apt.AP_F32):
    g = apt.ap_grid_desc()
    g.dim = dim
    g.precision = prec
    for a in range(3):
        g.n[a] = n[a]
        g.dx[a] = dx
    return g


def _sp(n=1000, q=-1.0, m=1.0):
    s = apt.ap_species_desc()
    s.q, s.m, s.n = q, m, n
    return s


def test_query_layout_sizes():
    g = _grid()
    lay = apt.ap_query_layout(g, [_sp(2048)])
    assert lay.grid_bytes == 9 * 64 * 32 * 4
    assert lay.n_cells == 64 * 32
    assert lay.n_tiles == 2 * 4           # default 32 x 8 tiles
    assert lay.work_bytes > 2048 * 4 * 8
    g64 = _grid(prec=apt.AP_F64)
    assert apt.ap_query_layout(g64, [_sp(2048)]).grid_bytes == 9 * 64 * 32 * 8


@pytest.mark.parametrize("mut,msg", [
    (lambda g: setattr(g, "dim", 4), "dim"),
    (lambda g: (setattr(g, "dim", 1), g.n.__setitem__(2, 0)), "rows"),
    (lambda g: (setattr(g, "dim", 1), g.dx.__setitem__(2, -0.5)), "row spacing"),
    (lambda g: setattr(g, "precision", 7), "precision"),
    (lambda g: g.n.__setitem__(0, 2), "4 cells"),
    (lambda g: g.dx.__setitem__(2, -1.0), "dx"),
    (lambda g: setattr(g, "dt", 0.2), "stability"),
    (lambda g: setattr(g, "dt", float("nan")), "dt"),
    (lambda g: (g.n.__setitem__(0, 256), g.tile.__setitem__(0, 100)), "tile"),
    (lambda g: setattr(g, "options", 0x40), "option"),
])
def test_query_layout_rejects_bad_grid(mut, msg):
    g = _grid()
    mut(g)
    with pytest.raises(apt.APTError) as ei:
        apt.ap_query_layout(g, [_sp()])
    assert ei.value.status == apt.AP_E_ARG
    assert msg in apt.last_error()


def test_query_layout_rejects_bad_species():
    with pytest.raises(apt.APTError):
        apt.ap_query_layout(_grid(), [_sp(m=0.0)])
    with pytest.raises(apt.APTError):
        apt.ap_query_layout(_grid(), [_sp(n=-5)])
    with pytest.raises(apt.APTError):
        apt.ap_query_layout(_grid(), [_sp()] * 5)


def test_gridless_layout_needs_dt():
    g = _grid(dim=0)
    with pytest.raises(apt.APTError):
        apt.ap_query_layout(g, [_sp()])
    g.dt = 0.01
    lay = apt.ap_query_layout(g, [_sp()])
    assert lay.grid_bytes == 0


def test_init_rejects_null_buffers_before_device_work():
    lib = apt.load()
    g = _grid()
    sp = (apt.ap_species_desc * 1)(_sp(16))
    bufs = apt.ap_buffers()
    ctx = C.c_void_p()
    st = lib.ap_init(C.byref(g), sp, 1, C.byref(bufs), None, C.byref(ctx))
    assert st == apt.AP_E_ARG and ctx.value is None
    assert "NULL" in apt.last_error()


def test_calls_on_null_context():
    lib = apt.load()
    assert lib.ap_step(None, 1, 0) == apt.AP_E_ARG
    assert lib.ap_set_pulse(None, 0, None) == apt.AP_E_ARG
    assert lib.ap_destroy(None) == apt.AP_OK
    d = apt.ap_diag()
    assert lib.ap_gather_diag(None, 1, C.byref(d)) == apt.AP_E_ARG


def test_pulse_on_grid_option_reserves_workspace():
    g = _grid()
    base = apt.ap_query_layout(g, [_sp(2048)]).work_bytes
    g.options = apt.AP_GRID_PULSE_ON_GRID
    more = apt.ap_query_layout(g, [_sp(2048)]).work_bytes
    assert more >= base + 6 * 64 * 32 * 4
    g0 = _grid(dim=0)
    g0.dt = 0.01
    g0.options = apt.AP_GRID_PULSE_ON_GRID
    with pytest.raises(apt.APTError):
        apt.ap_query_layout(g0, [_sp()])


def test_proxy_option_reserves_workspace():
    """AP_GRID_PROXY reserves the re-sort copy of each species' (sum,
    compensation) pairs; gridless runs reject the bit (they always take one)."""
    g = _grid()
    base = apt.ap_query_layout(g, [_sp(2048)]).work_bytes
    g.options = apt.AP_GRID_PROXY
    more = apt.ap_query_layout(g, [_sp(2048)]).work_bytes
    assert more >= base + 2 * 2048 * 4
    g0 = _grid(dim=0)
    g0.dt = 0.01
    g0.options = apt.AP_GRID_PROXY
    with pytest.raises(apt.APTError, match="AP_GRID_PROXY"):
        apt.ap_query_layout(g0, [_sp()])


def test_open_x_option_rows_only():
    """AP_GRID_OPEN_X needs a grid; gridded runs take it and reserve the
    per-row boundary source."""
    g = _grid(dim=0)
    g.dt = 0.01
    g.options = apt.AP_GRID_OPEN_X
    with pytest.raises(apt.APTError, match="needs a grid"):
        apt.ap_query_layout(g, [_sp()])
    g2 = _grid()
    g2.options = apt.AP_GRID_OPEN_X
    assert apt.ap_query_layout(g2, [_sp()]).work_bytes > 0
    g1 = _grid(dim=1)
    base = apt.ap_query_layout(g1, [_sp()]).work_bytes
    g1.options = apt.AP_GRID_OPEN_X
    assert apt.ap_query_layout(g1, [_sp()]).work_bytes >= base


def test_moving_window_option():
    """AP_GRID_MOVING_WINDOW reserves the shift's workspace on grids (the free-id
    bit map, its word popcounts and their scan, in 2-D the list of slots
    injected since the last sort: no copy of the fields) and is rejected
    without a grid or together with AP_GRID_OPEN_X."""
    g = _grid()
    base = apt.ap_query_layout(g, [_sp(2048)]).work_bytes
    g.options = apt.AP_GRID_MOVING_WINDOW
    extra = apt.ap_query_layout(g, [_sp(2048)]).work_bytes - base
    assert 3 * 64 * 4 <= extra < 6 * 64 * 32 * 4
    g0 = _grid(dim=0)
    g0.dt = 0.01
    g0.options = apt.AP_GRID_MOVING_WINDOW
    with pytest.raises(apt.APTError, match="moving window"):
        apt.ap_query_layout(g0, [_sp()])
    g.options = apt.AP_GRID_MOVING_WINDOW | apt.AP_GRID_OPEN_X
    with pytest.raises(apt.APTError, match="exclude each other"):
        apt.ap_query_layout(g, [_sp()])


def test_window_calls_on_null_context():
    lib = apt.load()
    assert lib.ap_shift_window(None, 1, None) == apt.AP_E_ARG
    assert lib.ap_get_window(None, None, None) == apt.AP_E_ARG
    d = C.c_int32()
    assert lib.ap_window_due(None, 1.0, 0.0, 0.0, C.byref(d)) == apt.AP_E_ARG


def test_library_has_no_unresolved_internal_symbols():
    """Every kernel launcher the library calls is instantiated in it (a
    missing template instantiation would only fail when loaded)."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--undefined-only", apt.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    bad = [ln for ln in out.splitlines() if "_ZN3apt" in ln or " ap_" in ln]
    assert not bad, bad


def test_pulse_params_struct_matches_header():
    """ap_pulse_params in the binding has the header's layout: 16 doubles, 10
    int32 (d_f ... no_fd), then fwhm, wp2, zeta."""
    assert C.sizeof(apt.ap_pulse_params) == 16 * 8 + 10 * 4 + 3 * 8
    assert apt.ap_pulse_params.fwhm.offset == 16 * 8 + 10 * 4
    assert apt.ap_pulse_params.zeta.offset == 16 * 8 + 10 * 4 + 16
    p = apt.pulse_params(envelope="sgauss", sampling="grid", fwhm=30.0)
    assert (p.envelope, p.sampling, p.fwhm) == (apt.AP_ENV_SGAUSS, apt.AP_SAMPLE_GRID, 30.0)
    q = apt.pulse_params(dispersion=apt.AP_DISP_PLASMA, wp2=0.05, fd=False)
    assert (q.wp2, q.zeta, q.no_fd) == (0.05, 0.0, 1)


def test_rows1d_layout():
    """dim 1: rows of 1-D lines; tiles along x only, one tile row per grid row."""
    g = _grid()
    g.dim = 1
    g.n[0], g.n[1], g.n[2] = 100, 7, 3
    g.dx[2] = 0.0
    lay = apt.ap_query_layout(g, [_sp()])
    assert lay.n_cells == 300
    assert lay.n_tiles == 4 * 3                  # default 32-cell tiles
    assert lay.grid_bytes == 9 * 300 * lay.real_bytes


def test_revolve_plan_is_the_optimal_binomial_schedule():
    """ap_revolve_plan's forward steps equal the optimum over every split,
    found by dynamic programming: C(n, s) = min_d d + C(n - d, s - 1) + C(d, s)
    (store the state d steps ahead, reverse the right part with one slot
    less, then the left part again from the start), C(1, s) = 0,
    C(n, 0) = n (n - 1) / 2; the recording sweep's first descent is free:
    F(n, s) = min_d F(n - d, s - 1) + C(d, s).  The repetitions bound the
    re-advancing: forward steps <= repetitions x n."""
    import functools

    @functools.lru_cache(maxsize=None)
    def cost(n, s):
        if n <= 1:
            return 0
        if s == 0:
            return n * (n - 1) // 2
        return min(d + cost(n - d, s - 1) + cost(d, s) for d in range(1, n))

    @functools.lru_cache(maxsize=None)
    def first(n, s):
        if n <= 1:
            return 0
        if s == 0:
            return cost(n, 0)
        return min(first(n - d, s - 1) + cost(d, s) for d in range(1, n))

    for slots in range(1, 7):
        for n in range(1, 61):
            t, f = apt.ap_revolve_plan(n, slots)
            assert f == first(n, slots - 1), (n, slots, f, first(n, slots - 1))
            assert f <= t * n and (t == 0) == (f == 0)
    # one slot: every step re-advanced from the start
    assert apt.ap_revolve_plan(10, 1) == (9, 45)
    # at scale: 20000 steps with 64 slots re-advance each step at most twice
    t, f = apt.ap_revolve_plan(20000, 64)
    assert t == 2 and f <= 2 * 20000
    with pytest.raises(apt.APTError):
        apt.ap_revolve_plan(0, 4)
