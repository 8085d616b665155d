"""Moving window (Sec. III.C) on the HIP path vs the oracle.

A 2-D LG replica (32 x 16 cells, electrons and protons, u x5, spare slots for
a quarter of the particles), 1-D LG rows (64 cells x 3 rows) and a 3-D
Gaussian replica (16 x 10 x 8) advance 24 steps with the window shifted
every 4 steps along +x or -x; each shift injects a fresh column of plasma
(``inputs.window_column``, its own seed) into the entering column.  Then a
flying focus (beta_f = -1 and 1.5) on an (x, z) replica whose window follows
the focus, scheduled from v_f by ap_window_due on the GPU and by
``pic.window_due`` in the oracle run.  Fields (ring origin undone) and, by
particle id, the live particles' cells, offsets and momenta match the
oracle's run (FP64, 1e-10 of the largest); free slots match its free ids.
Error paths: a run without the option, a direction other than +-1, injected
particles outside the entering column, more injected particles than free
slots.
"""
import numpy as np
import pytest
import torch

from oracle import pic, pulses, units
from paper_2307_04843_amd import apt, inputs
from tests import cases

pytestmark = pytest.mark.gpu

N_STEPS, EVERY = 24, 4
L = units.LAMBDA


def _pad(case):
    for sp in case["species"]:
        N = sp["state"]["w"].shape[0]
        sp["state"] = inputs.pad_free(sp["state"], N // 4, N)
    return case


def _setup(dim):
    if dim == 2:
        case = cases.make_case(n=(32, 1, 16), seed=81, u_scale=5.0, ppc=2)
    elif dim == 3:
        dxl = 0.0625
        n = (16, 10, 8)
        dt = units.default_dt(dxl, 3)
        box = tuple(nn * dxl for nn in n)
        pp = dict(type="gauss", a0=3.0, tau=20.0, x_ref=box[0] / 2, t_ref=10.0, x_f=box[0] / 2 + 0.3, w0=1.0,
                  y_c=box[1] / 2, z_c=box[2] / 2, d_f=3, pol=1, dispersion=units.DISP_PAPER2, dx_prop=dxl,
                  dt_prop=dt, dt=dt)
        case = cases.make_case(dim=3, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(10.0 / dt), ppc=2,
                               pulse=pp, u_scale=5.0, seed=83)
    else:
        case = cases.make_case(dim=1, n=(64, 1, 3), seed=82, u_scale=5.0, ppc=2, x_min=(48.0, 0.0, 4.4),
                               t0_steps=1343)
    return _pad(case)


def _column(case, shift, x_min_new, direction):
    dim, n = case["dim"], case["n"]
    out = []
    for i, sp in enumerate(case["species"]):
        col = inputs.window_column(dim, n, case["dx"], x_min_new, 2, inputs.density_uniform(0.02), 0.0,
                                   abs(sp["m"]), 900 + 10 * shift + i, column=n[0] - 1 if direction > 0 else 0)
        out.append(col)
    return out


def _oracle_species(case):
    dim, n = case["dim"], case["n"]
    nx, ny = n[0], (n[1] if dim == 3 else 1)
    sps = []
    for sp in case["species"]:
        st = sp["state"]
        cell = st["cell"].astype(np.int64)
        live = cell >= 0
        pos = np.zeros((3, live.sum()))
        c = cell[live]
        pos[0] = c % nx + st["off"][0][live].astype(float)
        if dim == 3:
            pos[1] = (c // nx) % ny + st["off"][1][live].astype(float)
        pos[2] = c // (nx * ny) + (st["off"][2][live].astype(float) if dim >= 2 else 0.0)
        ids = np.arange(cell.size)
        sps.append(pic.Species(sp["q"], sp["m"], pos, st["u"][:, live].astype(float), st["w"][live].astype(float),
                               ids=ids[live], free=ids[~live]))
    return sps


def _col_for_oracle(case, col):
    dim, n = case["dim"], case["n"]
    nx, ny = n[0], (n[1] if dim == 3 else 1)
    c = col["cell"].astype(np.int64)
    pos = np.zeros((3, c.size))
    pos[0] = c % nx + col["off"][0].astype(float)
    if dim == 3:
        pos[1] = (c // nx) % ny + col["off"][1].astype(float)
    pos[2] = c // (nx * ny) + (col["off"][2].astype(float) if dim >= 2 else 0.0)
    return pos, col["u"].astype(float), col["w"].astype(float)


def _oracle_grid(case):
    n = case["n"]
    g = pic.Grid(case["dim"], n, tuple(d * L for d in case["dx"]), case["dt"] * L,
                 tuple(v * L for v in case["x_min"]), t0=case["t0"] * L)
    for k in range(3):
        g.E[k][...] = case["fields"][k].astype(float)
        g.B[k][...] = case["fields"][3 + k].astype(float)
    return g


def _compare(case, sim, g, sps, x_min_expect):
    dim = case["dim"]
    out = [sim.state(i) for i in range(len(sps))]
    E, B = sim.window_fields()
    gf = [t.double().cpu().numpy() for t in E + B]
    d, _ = sim.diag()
    x_min, origin = sim.window()
    assert abs(x_min - x_min_expect) <= 1e-12 * max(1.0, abs(x_min_expect))
    assert abs(g.x_min[0] / L - x_min) <= 1e-12 * max(1.0, abs(x_min))
    fmax = max(np.abs(c).max() for c in g.E + g.B)
    for k in range(3):
        assert np.abs(gf[k] - g.E[k]).max() <= 1e-10 * fmax, ("E", k)
        assert np.abs(gf[3 + k] - g.B[k]).max() <= 1e-10 * fmax, ("B", k)
    assert d.n_nonfinite == 0
    for sp, st in zip(sps, out):
        live = st["cell"] >= 0
        assert np.array_equal(np.sort(st["id"][live]), np.sort(sp.ids))
        assert np.array_equal(np.sort(st["id"][~live]), np.sort(sp.free))
        order = np.argsort(sp.ids)
        o2 = np.argsort(st["id"][live])
        pos = cases.gpu_positions(case, {"cell": st["cell"][live], "off": st["off"][:, live]})
        for ax in (0, 1, 2) if dim == 3 else (0, 2):
            assert np.abs(pos[ax][o2] - sp.pos[ax][order]).max() <= 1e-10, ax
        assert np.abs(st["u"][:, live][:, o2] - sp.u[:, order]).max() <= 1e-10 * max(np.abs(sp.u).max(), 1.0)
    return origin


@pytest.mark.timeout(300)
@pytest.mark.parametrize("direction", [1, -1])
@pytest.mark.parametrize("dim", [2, 1, 3])
def test_moving_window_matches_oracle_fp64(dim, direction):
    case = _setup(dim)
    print("moving window, dim", dim, "direction", direction, flush=True)
    g = _oracle_grid(case)
    sps = _oracle_species(case)
    P = pulses.Pulse(case["pulse"])
    sim = cases.sim_from_case(case, precision="f64", sort_every=3, moving_window=True)
    try:
        x_min = list(case["x_min"])
        shift = 0
        for k in range(N_STEPS):
            if k % EVERY == EVERY - 1:
                x_min[0] += direction * case["dx"][0]
                cols = _column(case, shift, x_min, direction)
                sim.shift_window(cols, direction)
                pic.shift_window(g, sps, [_col_for_oracle(case, c) for c in cols], direction)
                shift += 1
            sim.step(1)
            pic.step(g, sps, P)
        origin = _compare(case, sim, g, sps, x_min[0])
    finally:
        sim.close()
    assert shift == N_STEPS // EVERY
    assert origin == (direction * shift) % case["n"][0]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("pattern", ["forward", "alternate"])
def test_window_2d_leavers_by_tile_ranges_fp64(pattern):
    """2-D run with 8 x 8 tiles (four tile columns) and a re-sort every 3
    steps: between sorts each shift finds its leavers in the slot ranges of
    the tile columns within reach since the sort, plus the particles injected
    since.  "alternate" shifts +x then -x in turn, so each shift's injected
    particles leave at the next one; those are found only through the list
    of injected slots.  Matches the oracle as above."""
    case = _setup(2)
    print("moving window, tile ranges,", pattern, flush=True)
    g = _oracle_grid(case)
    sps = _oracle_species(case)
    P = pulses.Pulse(case["pulse"])
    sim = cases.sim_from_case(case, precision="f64", sort_every=3, moving_window=True, tile=(8, 1, 8))
    try:
        x_min = list(case["x_min"])
        shift = 0
        for k in range(N_STEPS):
            if k % 2 == 1:
                direction = 1 if (pattern == "forward" or shift % 2 == 0) else -1
                x_min[0] += direction * case["dx"][0]
                cols = _column(case, shift, x_min, direction)
                sim.shift_window(cols, direction)
                pic.shift_window(g, sps, [_col_for_oracle(case, c) for c in cols], direction)
                shift += 1
            sim.step(1)
            pic.step(g, sps, P)
        _compare(case, sim, g, sps, x_min[0])
    finally:
        sim.close()
    assert shift == N_STEPS // 2


def _ff_window_case(beta_f):
    dxl = 0.05
    n = (40, 1, 20)
    dt = units.default_dt(dxl, 2)
    t0 = 10.0
    box = (n[0] * dxl, 0.0, n[2] * dxl)
    pp = dict(type="ff", a0=2.0, tau=40.0, x_ref=box[0] / 2, t_ref=t0, x_f=0.0, w0=0.5, y_c=0.0,
              z_c=box[2] / 2, d_f=2, pol=0, beta_f=beta_f, x0_ff=box[0] / 2, t0_ff=t0, chirp=0.05,
              dispersion=units.DISP_PAPER2, dx_prop=dxl, dt_prop=dt, dt=dt)
    case = cases.make_case(dim=2, n=n, dxl=dxl, x_min=(0.0, 0.0, 0.0), t0_steps=int(t0 / dt), ppc=2, pulse=pp,
                           u_scale=5.0, seed=91)
    return _pad(case)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("beta_f", [-1.0, 1.5])
def test_flying_focus_in_window_following_v_f(beta_f):
    """The window follows the focus at v_f = beta_f c (x_min anchored so that
    the focus stays at the window's centre); shifts come from ap_window_due
    on the GPU side and pic.window_due on the oracle side, with a plasma
    column injected on entry."""
    case = _ff_window_case(beta_f)
    g = _oracle_grid(case)
    sps = _oracle_species(case)
    P = pulses.Pulse(case["pulse"])
    x_ref, t_ref = case["x_min"][0], case["t0"]
    steps = 30
    shifts = {"n": 0}

    def inject(direction, x_min_new):
        cols = _column(case, shifts["n"], [x_min_new, 0.0, case["x_min"][2]], direction)
        shifts["n"] += 1
        return cols

    sim = cases.sim_from_case(case, precision="f64", sort_every=3, moving_window=True)
    try:
        net = sim.step_window(steps, beta_f, x_ref, t_ref, inject)
        n_gpu = shifts["n"]
        # the oracle run, scheduled from v_f in its own units
        shifts["n"] = 0
        net_o = 0
        for _ in range(steps):
            while True:
                d = pic.window_due(g.x_min[0], g.dx[0], g.t, beta_f, x_ref * L, t_ref * L)
                if d == 0:
                    break
                x_new = g.x_min[0] / L + d * case["dx"][0]
                cols = inject(d, x_new)
                pic.shift_window(g, sps, [_col_for_oracle(case, c) for c in cols], d)
                net_o += d
            pic.step(g, sps, P)
        assert shifts["n"] == n_gpu and net_o == net
        # the window moved with the focus: shifts are taken before each step,
        # the last at t0 + (steps - 1) dt, to within [-1/2, 1/2) cell
        expect = beta_f * (steps - 1) * case["dt"] / case["dx"][0]
        assert -0.5 <= expect - net < 0.5 and abs(net) >= 10
        _compare(case, sim, g, sps, x_ref + net * case["dx"][0])
    finally:
        sim.close()


def test_moving_window_errors():
    case = _setup(2)
    sim = cases.sim_from_case(case, precision="f64")
    try:
        with pytest.raises(apt.APTError, match="AP_GRID_MOVING_WINDOW"):
            sim.shift_window()
    finally:
        sim.close()
    sim = cases.sim_from_case(case, precision="f64", moving_window=True)
    try:
        x_min = list(case["x_min"])
        x_min[0] += case["dx"][0]
        cols = _column(case, 0, x_min, 1)
        with pytest.raises(apt.APTError, match="dir must be"):
            sim.shift_window(cols, 2)
        bad = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in cols[0].items()}
        bad["cell"] = bad["cell"] - 1          # not the entering column
        with pytest.raises(apt.APTError, match="entering column"):
            sim.shift_window([bad, None])
        # a -x shift takes its particles in the first column, not the last
        with pytest.raises(apt.APTError, match="entering column"):
            sim.shift_window(cols, -1)
        many = {k: np.concatenate([v] * 40, axis=-1) for k, v in cols[0].items()}
        with pytest.raises(apt.APTError, match="free slots"):
            sim.shift_window([many, None])
        # nothing changed: a valid shift still works and the run steps on
        assert sim.window() == (case["x_min"][0], 0)
        sim.shift_window(cols)
        sim.step(2)
        d, _ = sim.diag()
        assert d.n_nonfinite == 0
        assert sim.window()[1] == 1
    finally:
        sim.close()
