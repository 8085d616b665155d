"""Throughput of the analytic-pulse PIC hot path on one MI355X.

Headline (``value``): 3-D PIC, 1024 x 512 x 512 cells at lambda/16, c dt/dx =
0.95/sqrt(3), 2 electrons + 2 protons (m = 1836) per cell = 1.07e9 particles
in a Gaussian density channel n = 0.01 exp(-r^2/(20 lambda)^2) n_c, T = 1 eV;
analytic paraxial Gaussian pulse (D_f = 3, a0 = 3, w0 = 10 lambda, 30 lambda/c
sin^2 envelope, focus at the box centre, front at x = 0 at t = 0); FP32
particles and grid with an FP64 laser phase.  The particles are drawn on the
GPU.  The timed window is the END of the 1000-step run, where the pulse is
inside the plasma: the run starts at step 1000 - warmup - steps, takes
``--warmup`` untimed steps, then ``--steps`` timed ones.  One step = tile
sort + J clear + fused gather/analytic/Boris/move/Esirkepov kernel + J
rounding + Yee update.  ``value`` = particle pushes per second over the timed
steps, inputs resident in HBM.  The same window then runs in FP64
(``fp32_over_fp64``).  ``roofline`` is the fused kernel's algorithmic HBM
rate from its HIP-event launch time; ``cpu_baseline`` the FP64 oracle on a
16^3-cell replica inside the pulse at the window's clock.

Other legs (``--legs``):
  pic2d    the 4096 x 1024 LG run (16 e + 16 p per cell, 134M, 0 -> 0.05 n_c
           ramp, LG l=1 p=0 a0=5 w0=8 tau=30): the last steps of its 2000-step
           run in FP32 and FP64, with the grid-sampled pulse and with the
           analytic current, the moving-window shift cost, and a 512 x 1024
           box that lies inside the LG envelope for the whole window;
  adjoint  the gridless head-on collision (2^24 electrons, gamma = 2000, eps^4
           nonparaxial Gaussian a0 = 20, w0 = 2): forward with recording plus
           ap_backward for d<p_perp^2>/d(a0, w0, x_f), FP32 and FP64;
  adjoint_full  the same collision's whole 20000-step run under binomial
           checkpointing (64 whole states);
  three_d  the 512 x 256 x 256 flying-focus run (268M electrons, beta_f = -1,
           chirp 5%): steps 1800 ... 1900 of 4000, then the frozen-grid and the
           fully coupled adjoints over a 32-step window;
  small    the 128 x 64 Gaussian run (32768 electrons, 200 steps), FP64, FP32;
  rows1d   30 independent 1-D rows (Sec. III.B), 7.9M electrons, 500 steps;
  cpu      the oracle baselines.
Optional leg: adjoint3d_long, the 3-D run's frozen-grid adjoint over a
1000-step window under binomial checkpointing (16 whole states).

Prints one JSON line.  ``--gpus`` above 1 is refused (one GPU only).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LAMBDA_DX = 0.05
N_CELLS = (4096, 1, 1024)
PPC = 16


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def workload_inputs(n_cells=N_CELLS, x_min=(0.0, 0.0, -25.6), seed=2):
    """Electrons + protons of the 4096 x 1024 LG run (16 + 16 per cell), drawn
    on the GPU (``inputs.plasma_device``)."""
    return pic2d_inputs(n_cells, x_min, seed)


def workload_pulse(dt):
    """LG l=1 p=0 pulse parameters (lambda units) for the 4096 x 1024 box."""
    dx = LAMBDA_DX
    c2 = (dt / dx) ** 2
    kdx = 2 * math.pi * dx
    vg = 1.0 - (1.0 - c2) * kdx ** 2 / 8.0          # second-order group velocity
    x_f = N_CELLS[0] * dx / 2
    tau = 30.0
    return dict(a0=5.0, tau=tau, x_ref=x_f, t_ref=tau / 2 + x_f / vg, x_f=x_f, w0=8.0, y_c=0.0, z_c=0.0,
                q_slice=0.0, d_f=3, lg_l=1, lg_p=0, pol=1, dispersion=0, dx_prop=dx, dt_prop=dt)


N3 = (512, 256, 256)
DX3 = 0.0625
PPC3 = 8
T0_STEP3 = 1800


def workload3d_inputs(seed=4):
    from paper_2307_04843_amd import inputs
    e = inputs.plasma(3, N3, (DX3,) * 3, (0.0, -8.0, -8.0), PPC3, inputs.density_uniform(0.001), 1.0, 1.0,
                      seed, stream=0)
    return [dict(q=-1.0, m=1.0, state=e)]


def workload3d_pulse(dt):
    """Flying focus for the 512 x 256 x 256 box: front at x = 0 at t = 0, focus
    moving backwards at c through the box centre at step 1850."""
    c2 = (dt / DX3) ** 2
    kdx = 2 * math.pi * DX3
    vg = 1.0 - (1.0 - c2) * kdx ** 2 / 8.0
    xc = N3[0] * DX3 / 2
    tau = 150.0
    return dict(a0=2.0, tau=tau, x_ref=xc, t_ref=tau / 2 + xc / vg, x_f=0.0, w0=4.0, y_c=0.0, z_c=0.0, d_f=3,
                pol=0, beta_f=-1.0, x0_ff=xc, t0_ff=(T0_STEP3 + 50) * dt, chirp=0.05, dispersion=0,
                dx_prop=DX3, dt_prop=dt)


def three_d_leg(args):
    import torch
    from paper_2307_04843_amd import apt
    from paper_2307_04843_amd.autograd import APTRun, GriddedRun
    from paper_2307_04843_amd.sim import Simulation
    log("3-D: generating inputs")
    species = workload3d_inputs()
    n = int(species[0]["state"]["u"].shape[1])
    dt = 0.95 / math.sqrt(3) * DX3
    t0 = T0_STEP3 * dt
    pp = workload3d_pulse(dt)
    geo = dict(n=N3, dx=(DX3,) * 3, x_min=(0.0, -8.0, -8.0), t0=t0, dt=dt)
    out = {"workload": "3-D PIC 512x256x256 cells lambda/16, 8 e per cell (268M), 0.001 n_c, immobile "
                       "ions, flying focus beta_f=-1 a0=2 w0=4 tau=150 chirp 5%%, steps %d..%d of the "
                       "4000-step run" % (T0_STEP3, T0_STEP3 + args.steps3d), "particles": n,
           "steps": args.steps3d, "warmup": 5}
    tile3 = tuple(int(v) for v in args.tile3.split(",")) if args.tile3 else (0, 0, 0)
    sim = Simulation(3, precision="f32", species=species, tile=tile3, **geo)
    try:
        sim.set_pulse("ff", **pp)
        sim.step(5)
        torch.cuda.synchronize()
        apt.ap_timing_enable(sim.ctx, True)
        apt.ap_timing_read(sim.ctx, reset=True)
        w0 = time.perf_counter()
        sim.step(args.steps3d)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        tm = apt.ap_timing_read(sim.ctx, reset=True)
        d, _ = sim.diag(allow_numeric=True)
        ms_push = tm.ms_push / max(1, tm.n_push)
        # particle bytes (read 32, write 28) + grid share (stage 24, flush 12 per cell)
        bl = n * 60 + sim.ncell * 36
        out.update({"pushes_per_s": n * args.steps3d / wall, "ms_per_step": wall * 1e3 / args.steps3d,
                    "push_ms_per_launch": ms_push, "hbm_gbs_algorithmic": bl / (ms_push * 1e-3) / 1e9,
                    "hbm_frac": bl / (ms_push * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "yee_ms": tm.ms_yee / max(1, tm.n_yee), "sort_ms_per_step": tm.ms_sort / args.steps3d,
                    "n_nonfinite": d.n_nonfinite, "n_fast": d.n_fast,
                    "offtile_fraction": d.n_offtile / float(n * (args.steps3d + 5))})
        log("3-D: %.3e pushes/s, push %.3f ms/launch" % (out["pushes_per_s"], ms_push))
    finally:
        sim.close()
        del sim
        torch.cuda.empty_cache()
    if args.adj3d_steps > 0:
        names = ["beta_f", "chirp"]
        K = 8
        for coupled in (False, True) if not args.skip_coupled else (False,):
            key = "adjoint_coupled" if coupled else "adjoint"
            log("3-D %s: %d-step window, segments of %d" % (key, args.adj3d_steps, K))
            run = GriddedRun(3, N3, (DX3,) * 3, (0.0, -8.0, -8.0), species, "ff", pp, names, args.adj3d_steps,
                             t0=t0, dt=dt, precision="f32", segment=K, coupled=coupled)
            try:
                p = torch.tensor([pp["beta_f"], pp["chirp"]], dtype=torch.float64, requires_grad=True)
                torch.cuda.synchronize()
                free_gb = torch.cuda.mem_get_info()[0] / 1e9
                a = time.perf_counter()
                u, _ = APTRun.apply(p, run)
                torch.cuda.synchronize()
                b = time.perf_counter()
                obs = (u[1].double() ** 2 + u[2].double() ** 2).sum() / n
                obs.backward()
                torch.cuda.synchronize()
                c = time.perf_counter()
                note = ("fully coupled: every species' push, current, the Yee update and the gather "
                        "differentiated; backward = segment replays + transposed Yee + reverse steps" if coupled
                        else "frozen-grid reading; backward = segment replays with the full loop + reverse steps")
                out[key] = {"window_steps": args.adj3d_steps, "segment": K, "params": names,
                            "grad": p.grad.tolist(), "observable": float(obs.detach()),
                            "forward_pushes_per_s": n * args.adj3d_steps / (b - a),
                            "adjoint_pushes_per_s": n * args.adj3d_steps / (c - b),
                            "checkpoint_gb": run.ckpt.numel() / 1e9, "hbm_free_gb_at_forward": free_gb,
                            "note": note}
                log("3-D %s: %.3e pushes/s" % (key, out[key]["adjoint_pushes_per_s"]))
            finally:
                run.close()
                del run
                torch.cuda.empty_cache()
    del species
    return out


N5 = (1024, 512, 512)
X5_MIN = (0.0, -16.0, -16.0)
RUN5_STEPS = 1000   # length of the 1024 x 512 x 512 run


def large3d_inputs(seed=5, precision="f32"):
    """Electrons + protons of the 1024 x 512 x 512 channel (2 + 2 per cell,
    1.07e9 particles), drawn on the GPU (``inputs.plasma_device``)."""
    import torch
    from paper_2307_04843_amd import inputs
    dens = inputs.density_gauss_channel(0.01, 20.0, 0.0, 0.0)
    e = inputs.plasma_device(3, N5, (DX3,) * 3, X5_MIN, 2, dens, 1.0, 1.0, seed, stream=0)
    p = inputs.plasma_device(3, N5, (DX3,) * 3, X5_MIN, 2, dens, 1.0, inputs.PROTON_MASS, seed, stream=1,
                             positions_from=e)
    if precision == "f64":
        for st in (e, p):
            for key in ("off", "u", "w"):
                st[key] = st[key].to(torch.float64)
    return [dict(q=-1.0, m=1.0, state=e), dict(q=1.0, m=inputs.PROTON_MASS, state=p)]


def large3d_pulse(dt):
    """Gaussian (D_f = 3, a0 = 3, w0 = 10, tau = 30) focused at the centre of
    the 1024 x 512 x 512 box; its front is at x = 0 at t = 0."""
    c2 = (dt / DX3) ** 2
    vg = 1.0 - (1.0 - c2) * (2 * math.pi * DX3) ** 2 / 8.0
    xc = N5[0] * DX3 / 2
    return dict(a0=3.0, tau=30.0, x_ref=xc, t_ref=15.0 + xc / vg, x_f=xc, w0=10.0, y_c=0.0, z_c=0.0, d_f=3, pol=0,
                dispersion=0, dx_prop=DX3, dt_prop=dt)


def window_start(run_steps, warmup, steps):
    """First step of a window of warmup + steps steps that ends at the end of
    the run: the pulse is then inside the plasma for the whole window."""
    return max(0, run_steps - warmup - steps)


def large3d_run(precision, warmup, steps, timing=True, tile=(0, 0, 0)):
    """The last warmup + steps steps of the 1000-step 1024 x 512 x 512 run:
    `warmup` untimed, then `steps` timed between synchronisations."""
    import torch
    from paper_2307_04843_amd import apt
    from paper_2307_04843_amd.sim import Simulation
    log("large 3-D %s: generating 1.07e9 particles on the GPU" % precision)
    a = time.perf_counter()
    species = large3d_inputs(precision=precision)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - a
    n = sum(int(s["state"]["u"].shape[1]) for s in species)
    dt = 0.95 / math.sqrt(3) * DX3
    s0 = window_start(RUN5_STEPS, warmup, steps)
    sim = Simulation(3, n=N5, dx=(DX3,) * 3, x_min=X5_MIN, t0=s0 * dt, dt=dt, precision=precision,
                     species=species, tile=tile)
    del species
    try:
        sim.set_pulse("gauss", **large3d_pulse(dt))
        sim.step(warmup)
        torch.cuda.synchronize()
        if timing:
            apt.ap_timing_enable(sim.ctx, True)
            apt.ap_timing_read(sim.ctx, reset=True)
        a = time.perf_counter()
        done = 0
        while done < steps:
            k = min(25, steps - done)
            sim.step(k)
            done += k
            if done < steps:
                torch.cuda.synchronize()   # a progress line every 25 steps
                log("large 3-D %s: %d/%d steps, %.1f s" % (precision, done, steps, time.perf_counter() - a))
        torch.cuda.synchronize()
        wall = time.perf_counter() - a
        tm = apt.ap_timing_read(sim.ctx, reset=True) if timing else None
        d, st = sim.diag(allow_numeric=True)
        return dict(wall=wall, n_part=n, ncell=sim.ncell, timing=tm, diag=d, status=st, first_step=s0,
                    gen_s=gen_s)
    finally:
        sim.close()
        del sim
        torch.cuda.empty_cache()


def rows1d_leg():
    import torch
    from paper_2307_04843_amd import apt, inputs
    from paper_2307_04843_amd.sim import Simulation
    dx = 0.05
    n = (4096, 1, 30)
    dt = 0.95 * dx
    e = inputs.plasma(1, n, (dx, dx, 0.1), (0.0, 0.0, 0.0), 64, inputs.density_uniform(0.01), 1.0, 1.0, 7)
    npart = int(e["u"].shape[1])
    vg = 1.0 - (1.0 - (dt / dx) ** 2) * (2 * math.pi * dx) ** 2 / 8.0
    pp = dict(a0=5.0, tau=10.0, x_ref=102.4, t_ref=5.0 + 102.4 / vg, x_f=102.4, w0=2.5, y_c=0.0, z_c=0.0, d_f=3,
              pol=0, dispersion=0, dx_prop=dx, dt_prop=dt)
    out = {"workload": "30 rows of 1-D PIC, 4096 cells lambda/20 each, rows 0.1 lambda apart, 64 e per cell "
                       "(7.9M), 0.01 n_c, Gaussian D_f=3 a0=5 w0=2.5 tau=10, 500 steps", "particles": npart,
           "steps": 500}
    sim = Simulation(1, n=n, dx=(dx, dx, 0.1), x_min=(0.0, 0.0, 0.0), t0=100.0, dt=dt, precision="f32",
                     species=[dict(q=-1.0, m=1.0, state=e)])
    try:
        sim.set_pulse("gauss", **pp)
        sim.step(5)
        torch.cuda.synchronize()
        apt.ap_timing_enable(sim.ctx, True)
        apt.ap_timing_read(sim.ctx, reset=True)
        a = time.perf_counter()
        sim.step(500)
        torch.cuda.synchronize()
        wall = time.perf_counter() - a
        tm = apt.ap_timing_read(sim.ctx, reset=True)
        d, _ = sim.diag(allow_numeric=True)
        out.update({"pushes_per_s": npart * 500 / wall, "ms_per_step": wall * 2.0,
                    "push_ms_per_launch": tm.ms_push / max(1, tm.n_push),
                    "n_nonfinite": d.n_nonfinite, "n_fast": d.n_fast})
    finally:
        sim.close()
    return out


def small_leg():
    """The 128 x 64 Gaussian run: 32768 electrons, 200 steps, FP64 and FP32."""
    import torch
    from paper_2307_04843_amd import inputs
    from paper_2307_04843_amd.sim import Simulation
    dx = 0.05
    dt = 0.95 / math.sqrt(2) * dx
    e = inputs.plasma(2, (128, 1, 64), (dx,) * 3, (0.0, 0.0, 0.0), 4, inputs.density_uniform(0.01), 1.0, 1.0,
                      1, stream=0)
    c2 = (dt / dx) ** 2
    vg = 1.0 - (1.0 - c2) * (2 * math.pi * dx) ** 2 / 8.0
    pp = dict(a0=1.0, tau=10.0, x_ref=3.2, t_ref=5.0 + 3.2 / vg, x_f=3.2, w0=5.0, y_c=0.0, z_c=1.6,
              q_slice=0.0, d_f=2, pol=1, dispersion=0, dx_prop=dx, dt_prop=dt)
    out = {"workload": "2-D PIC 128x64 cells lambda/20, 4 e per cell (32768), 0.01 n_c, immobile ions, "
                       "Gaussian D_f=2 a0=1 w0=5 tau=10, 200 steps", "particles": 32768, "steps": 200}
    for prec in ("f64", "f32"):
        sim = Simulation(2, n=(128, 1, 64), dx=(dx,) * 3, x_min=(0.0, 0.0, 0.0), t0=0.0, dt=dt, precision=prec,
                         species=[dict(q=-1.0, m=1.0, state=e)])
        try:
            sim.set_pulse("gauss", **pp)
            sim.step(5)
            torch.cuda.synchronize()
            a = time.perf_counter()
            sim.step(200)
            torch.cuda.synchronize()
            out[prec + "_pushes_per_s"] = 32768 * 200 / (time.perf_counter() - a)
        finally:
            sim.close()
    return out


RUN2_STEPS = 2000   # length of the 4096 x 1024 run


def run_gpu(species, precision, steps, warmup, timing=True, sort_every=0, on_grid=False, window_shifts=0,
            current=False, first_step=0, n_cells=N_CELLS, x_min=(0.0, 0.0, -25.6)):
    """The 4096 x 1024 LG run (or a box of it, n_cells at x_min) from step
    `first_step`: `warmup` untimed steps, then `steps` timed ones."""
    import torch
    from paper_2307_04843_amd import apt, inputs
    from paper_2307_04843_amd.sim import Simulation
    dt = 0.95 / math.sqrt(2) * LAMBDA_DX
    sim = Simulation(2, n=n_cells, dx=(LAMBDA_DX,) * 3, x_min=x_min, t0=first_step * dt, dt=dt,
                     precision=precision, species=species, sort_every=sort_every, pulse_on_grid=on_grid,
                     moving_window=window_shifts > 0)
    try:
        pp = workload_pulse(dt)
        if current:
            # Sec. IV: the pulse carries the analytic current of a 0.05 n_c plasma (J1 on the grid)
            pp.update(dispersion=3, wp2=0.05)
        sim.set_pulse("lg", **pp, sampling="grid" if on_grid else "particles")
        n_part = sum(int(s["state"]["u"].shape[1]) for s in species)
        sim.step(warmup)
        torch.cuda.synchronize()
        if timing:
            apt.ap_timing_enable(sim.ctx, True)
            apt.ap_timing_read(sim.ctx, reset=True)
        t0 = time.perf_counter()
        done = 0
        chunk = 250
        while done < steps:
            k = min(chunk, steps - done)
            sim.step(k)
            done += k
            if done < steps:
                torch.cuda.synchronize()   # one sync per chunk: a progress line, negligible cost
                log("%s: %d/%d steps, %.1f s" % (precision, done, steps, time.perf_counter() - t0))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tm = apt.ap_timing_read(sim.ctx, reset=True) if timing else None
        d, st = sim.diag(allow_numeric=True)
        shift_ms = None
        if window_shifts > 0:
            # after the timed run: the moving window (Sec. III.C) advanced one
            # cell at a time between steps, each shift injecting the entering
            # column's plasma (1 e + 1 p per cell, resident on the GPU before
            # the clock starts); the first shifts free the slots of the
            # particles left behind.  Wall time of ap_shift_window alone.
            dens = inputs.density_ramp_x(0.05, 0.0, 200.0)
            x0 = sim.window()[0]
            walls = []
            for k in range(window_shifts):
                x_new = [x0 + (k + 1) * LAMBDA_DX, 0.0, x_min[2]]
                cols = None
                if k >= 2:
                    e = inputs.window_column(2, n_cells, (LAMBDA_DX,) * 3, x_new, 1, dens, 1.0, 1.0, 70 + k)
                    p = inputs.window_column(2, n_cells, (LAMBDA_DX,) * 3, x_new, 1, dens, 1.0,
                                             inputs.PROTON_MASS, 70 + k, stream=1)
                    p["cell"], p["off"] = e["cell"], e["off"]
                    cols = [{key: torch.as_tensor(v, device=sim.device) for key, v in c.items()} for c in (e, p)]
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                sim.shift_window(cols)
                torch.cuda.synchronize()
                walls.append(time.perf_counter() - t1)
                sim.step(1)
            shift_ms = 1e3 * sum(walls[2:]) / max(1, len(walls) - 2)
        return dict(wall=wall, n_part=n_part, timing=tm, diag=d, status=st, ncell=sim.ncell, shift_ms=shift_ms)
    finally:
        sim.close()


def _oracle_species(st, n, q_m):
    """Oracle species (positions in cell units) from an inputs.plasma state."""
    import numpy as np
    from oracle import pic
    c = st["cell"].astype(np.int64)
    pos = np.zeros((3, c.size))
    pos[0] = c % n[0] + st["off"][0]
    pos[1] = (c // n[0]) % n[1] + st["off"][1]
    pos[2] = c // (n[0] * n[1]) + st["off"][2]
    return pic.Species(q_m[0], q_m[1], pos, st["u"].astype(float), st["w"].astype(float))


def cpu_baseline(first_step, budget_s=20.0):
    """The FP64 oracle on a bounded replica of the headline workload (host).

    Sample: a 16 x 16 x 16-cell periodic replica of the 1024 x 512 x 512 run
    at its resolution, 2 e + 2 p per cell (16384 particles) in the channel's
    density, around the laser axis at x = 16 ... 17 lambda with the clock at
    `first_step` (the first step of the timed window), so the Gaussian pulse
    covers it as it covers the timed steps; steps until ~budget_s of CPU
    time.  NumPy elementwise work runs on one core.
    """
    from oracle import pic, pulses, units
    from paper_2307_04843_amd import inputs
    L = units.LAMBDA
    n = (16, 16, 16)
    x_min = (16.0, -0.5, -0.5)
    dt = 0.95 / math.sqrt(3) * DX3
    dens = inputs.density_gauss_channel(0.01, 20.0, 0.0, 0.0)
    e = inputs.plasma(3, n, (DX3,) * 3, x_min, 2, dens, 1.0, 1.0, 6, stream=0)
    p = inputs.plasma(3, n, (DX3,) * 3, x_min, 2, dens, 1.0, inputs.PROTON_MASS, 6, stream=1, positions_from=e)
    g = pic.Grid(3, n, (DX3 * L,) * 3, dt * L, tuple(v * L for v in x_min), t0=first_step * dt * L)
    sps = [_oracle_species(e, n, (-1.0, 1.0)), _oracle_species(p, n, (1.0, inputs.PROTON_MASS))]
    pp = large3d_pulse(dt)
    P = pulses.Pulse(dict(type="gauss", dt=dt, **{k: v for k, v in pp.items() if k != "dt_prop"}))
    N = sum(s.pos.shape[1] for s in sps)
    steps = 0
    t0 = time.perf_counter()
    while True:
        pic.step(g, sps, P)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 200:
            break
    wall = time.perf_counter() - t0
    return dict(value=N * steps / wall, unit="pushes/s", cores=1, kind="oracle",
                sample="16x16x16-cell replica of the 1024x512x512 run at x = 16-17 lambda about the laser "
                       "axis, clock at step %d (the timed window, pulse present), %d particles (2 e + 2 p per "
                       "cell), %d steps, FP64 NumPy, single thread" % (first_step, N, steps))


def cpu_baseline_2d(budget_s=10.0):
    """The FP64 oracle on a 64 x 64-cell replica of the 4096 x 1024 LG run
    (16 e + 16 p per cell at x = 48-51.2 lambda, clock at step 1900, inside
    the pulse), one core."""
    from oracle import pic, pulses, units
    from paper_2307_04843_amd import inputs
    L = units.LAMBDA
    n = (64, 1, 64)
    x_min = (48.0, 0.0, 3.2)
    dt = 0.95 / math.sqrt(2) * LAMBDA_DX
    dens = inputs.density_ramp_x(0.05, 0.0, 200.0)
    e = inputs.plasma(2, n, (LAMBDA_DX,) * 3, x_min, PPC, dens, 1.0, 1.0, 6, stream=0)
    p = inputs.plasma(2, n, (LAMBDA_DX,) * 3, x_min, PPC, dens, 1.0, inputs.PROTON_MASS, 6, stream=1,
                      positions_from=e)
    g = pic.Grid(2, n, (LAMBDA_DX * L,) * 3, dt * L, tuple(v * L for v in x_min), t0=1900 * dt * L)
    sps = [_oracle_species(e, n, (-1.0, 1.0)), _oracle_species(p, n, (1.0, inputs.PROTON_MASS))]
    pp = workload_pulse(dt)
    P = pulses.Pulse(dict(type="lg", dt=dt, **{k: v for k, v in pp.items() if k != "dt_prop"}))
    N = sum(s.pos.shape[1] for s in sps)
    steps = 0
    t0 = time.perf_counter()
    while True:
        pic.step(g, sps, P)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 50:
            break
    wall = time.perf_counter() - t0
    return dict(value=N * steps / wall, unit="pushes/s", cores=1, kind="oracle",
                sample="64x64-cell replica of the 4096x1024 LG run at x=48-51.2 lambda, step 1900 clock, "
                       "%d particles, %d steps, FP64 NumPy, single thread" % (N, steps))


ADJ_N = 1 << 24
ADJ_T0 = 90.0
ADJ_DT = 0.01


def adjoint_beam(n=ADJ_N):
    from paper_2307_04843_amd import inputs
    return inputs.beam(n, 2000.0, 0.05, 1.0, 1.0, 10.0, 1.0, seed=3)


def adjoint_pulse():
    return dict(a0=20.0, tau=20.0, t_ref=100.0, x_ref=0.0, x_f=0.0, w0=2.0, np_order=4,
                dispersion=2, pol=0)


def run_adjoint(beam, precision, steps, t0=ADJ_T0, revolve=None):
    """Forward (recording) + backward of the collision run; wall times and gradient."""
    import torch
    from paper_2307_04843_amd.autograd import APTRun, GridlessRun
    names = ["a0", "w0", "x_f"]
    vals = [20.0, 2.0, 0.0]
    run = GridlessRun(beam, "gauss_np", adjoint_pulse(), names, steps, ADJ_DT, t0=t0, precision=precision,
                      revolve=revolve)
    try:
        n = int(beam["u"].shape[1])
        p = torch.tensor(vals, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, _ = APTRun.apply(p, run)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        obs = (u[1].double() ** 2 + u[2].double() ** 2).sum() / n
        obs.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out = dict(forward_s=t1 - t0, backward_s=t2 - t1, grad=p.grad.tolist(), observable=float(obs.detach()),
                   forward_pushes_per_s=n * steps / (t1 - t0), adjoint_pushes_per_s=n * steps / (t2 - t1),
                   checkpoint_gb=run.ckpt.numel() / 1e9)
        if revolve:
            out["revolve_slots"] = revolve
        else:
            out["segment"] = run.segment
        return out
    finally:
        run.close()
        del run
        torch.cuda.empty_cache()


def _cpu_gridless_chunk(args):
    """Oracle gridless steps on one chunk of the sample, timed after a warm-up
    step (the oracle derives its eps^4 field functions on first use).
    Returns (pushes, seconds)."""
    X0, u0, steps = args
    from oracle import grad as ograd
    prm = dict(type="gauss_np", **adjoint_pulse())
    t_start = 99.0   # pulse and beam overlap: the expensive part of the run
    ograd.run_gridless(prm, X0[:, :64], u0[:, :64], -1.0, t_start, ADJ_DT, 1)
    t0 = time.perf_counter()
    ograd.run_gridless(prm, X0, u0, -1.0, t_start, ADJ_DT, steps)
    return X0.shape[1] * steps, time.perf_counter() - t0


def cpu_gridless_baseline(budget_s=8.0):
    """The FP64 oracle's gridless step (eps^4 field + Boris + move) on the host:
    one process, then one process per available core (at most 16; the run is
    embarrassingly parallel over particles)."""
    import multiprocessing as mp
    b = adjoint_beam(1 << 13)
    X0 = (b["icell"].astype(float) + b["off"].astype(float))
    u0 = b["u"].astype(float)
    n1, w1 = _cpu_gridless_chunk((X0, u0, 1))
    steps = max(1, int(budget_s / 2 / w1))
    n1, w1 = _cpu_gridless_chunk((X0, u0, steps))
    single = n1 / w1
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        res = pool.map(_cpu_gridless_chunk, [(X0, u0, steps)] * cores)
    multi = sum(r[0] for r in res) / max(r[1] for r in res)
    return dict(value=single, unit="pushes/s", cores=1, kind="oracle", all_core_value=multi,
                all_core_cores=cores,
                sample="8192 electrons of the collision beam from t = 99 lambda/c (inside the eps^4 "
                       "pulse), %d steps, FP64 NumPy; all-core: %d spawned processes on the same "
                       "sample, throughput = total pushes / slowest worker" % (steps, cores))


METRIC = "particle pushes/s (field eval+push+deposit) FP32 & adjoint vs FP64, 1 MI355X"

# Non-packed FP32 VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz.
VALU_PEAK_T_LANE_OPS = 256 * 4 * 16 * 2.4e9 / 1e12

PUSH3D_SOURCES = ("push3d.hip", "push3d_impl.h", "push3d_t844.hip", "kernels.h", "common.h", "pulse_dev.h",
                  "dual.h", "nonparaxial_gen.h", "apt_host.cpp")

# Counter measurements of k_push_deposit_3d on the headline window (this
# script's default --steps/--warmup), from rocprofv3 --pmc runs of it: HBM bytes per launch (FETCH_SIZE, WRITE_SIZE, each scaled by
# what the counter reads for a device copy of known size in the same run),
# VALU lane-ops per push (SQ_INSTS_VALU x 64 / pushes) and the LDS pipe's busy
# share.  Valid only for the kernel sources whose digest is recorded here.
MEASURED_TRAFFIC = {
    "sources_sha256": "5ee2c2cd7d37705b160ef32eab7d15f71fdf732db7b92eacf888cf2401ac31e1",
    # FETCH_SIZE 2.981e7 KiB x 1.99993 (a 2 GiB device copy reads as 1048610.8 KiB)
    "fetch_bytes_per_launch": 6.104e10,
    # WRITE_SIZE 7.640e7 KiB x 1.0 (the same copy writes as 2097152 KiB)
    "write_bytes_per_launch": 7.823e10,
    "valu_lane_ops_per_push": 1491.2,
    "ms_per_launch": 89.871,
    "lds_busy_frac": 0.503,
    "lds_bank_conflict_frac": 0.578,
    "note": "means over the 55 launches of the window, 2 GiB copy calibration in the same runs "
            "(profiles/push_deposit_3d_gauss_1024x512x512_f32.md)",
}


def sources_digest(names=PUSH3D_SOURCES):
    """SHA-256 over the sources that define the 3-D push kernel and its launch."""
    import hashlib
    d = os.path.join(ROOT, "paper_2307_04843_amd", "csrc")
    h = hashlib.sha256()
    for nm in names:
        h.update(nm.encode())
        with open(os.path.join(d, nm), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def headline_leg(args):
    """1024 x 512 x 512 run, 1.07e9 particles: the last warmup + steps steps of
    its 1000 steps, FP32 (FP64 phase island), then the same window in FP64."""
    tile3 = tuple(int(v) for v in args.tile3.split(",")) if args.tile3 else (0, 0, 0)
    r = large3d_run("f32", args.warmup, args.steps, tile=tile3)
    tm = r["timing"]
    n_part = r["n_part"]
    value = n_part * args.steps / r["wall"]
    ms_push = tm.ms_push / max(1, tm.n_push)
    # algorithmic bytes of one launch of the fused kernel: every particle read
    # (cell 4 + offsets 12 + u 12 + w 4 = 32 B) and written (cell 4 + offsets
    # 12 + u 12 = 28 B), plus the grid share (stage E2, B2: 24 B/cell; J flush 12 B/cell)
    bytes_launch = n_part * 60 + r["ncell"] * 36
    achieved = bytes_launch / (ms_push * 1e-3) / 1e9
    traffic = None
    traffic_note = "no counter measurement for the current kernel sources"
    roofline_valu = roofline_lds = None
    M = MEASURED_TRAFFIC
    if M is not None and M["sources_sha256"] == sources_digest():
        tb = M["fetch_bytes_per_launch"] + M["write_bytes_per_launch"]
        traffic = tb
        traffic_note = ("HBM bytes per launch (fetch %.4g + write %.4g) from rocprofv3 FETCH_SIZE/WRITE_SIZE, "
                        "%s" % (M["fetch_bytes_per_launch"], M["write_bytes_per_launch"], M["note"]))
        ops = M["valu_lane_ops_per_push"] * n_part / (M["ms_per_launch"] * 1e-3) / 1e12
        roofline_valu = {"bound": "alu", "achieved": ops, "peak": VALU_PEAK_T_LANE_OPS,
                         "unit": "T VALU lane-ops/s", "frac": ops / VALU_PEAK_T_LANE_OPS,
                         "per_push": M["valu_lane_ops_per_push"], "ms_per_launch": M["ms_per_launch"],
                         "note": "VALU lane-ops per push counted by rocprofv3 (SQ_INSTS_VALU) over the "
                                 "launch time of the same profiled runs, non-packed FP32 issue peak"}
        roofline_lds = {"bound": "lds", "busy_frac": M["lds_busy_frac"],
                        "bank_conflict_frac_of_busy": M["lds_bank_conflict_frac"],
                        "note": "share of the kernel's cycles in which the LDS pipe is busy "
                                "(rocprofv3 SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT), same window"}
    log("headline FP32: %.3e pushes/s, push %.3f ms/launch, yee %.3f ms, sort %.3f ms/step"
        % (value, ms_push, tm.ms_yee / max(1, tm.n_yee), tm.ms_sort / max(1, args.steps)))
    first = r["first_step"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3-D PIC 1024x512x512 cells lambda/16, c dt/dx 0.95/sqrt(3), 2 e + 2 p per cell "
                               "(1.07e9 particles, generated on the GPU), n = 0.01 exp(-r^2/(20 lambda)^2) n_c, "
                               "T = 1 eV, analytic paraxial Gaussian D_f=3 a0=3 w0=10 lambda tau=30 lambda/c "
                               "focused at the box centre, FP32 with an FP64 laser phase; timed steps %d..%d of "
                               "the 1000-step run (pulse inside the plasma)" % (first + args.warmup,
                                                                              first + args.warmup + args.steps),
                   "particles": n_part, "cells": r["ncell"], "first_timed_step": first + args.warmup},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_note": traffic_note,
                     "kernel": "k_push_deposit_3d", "ms_per_launch": ms_push,
                     "bytes_per_launch": bytes_launch,
                     "bytes_note": "60 B per particle (read cell, offsets, u, w; write cell, offsets, u) + 36 B "
                                   "per cell (stage E2, B2; flush J)"},
        "roofline_valu": roofline_valu,
        "roofline_lds": roofline_lds,
        "kernels_ms_per_step": {"push_deposit": ms_push, "yee": tm.ms_yee / max(1, tm.n_yee),
                                "sort": tm.ms_sort / max(1, args.steps),
                                "other": tm.ms_other / max(1, args.steps)},
        "numerics": {"n_nonfinite": r["diag"].n_nonfinite, "n_fast": r["diag"].n_fast,
                     "offtile_fraction": r["diag"].n_offtile / float(n_part * (args.steps + args.warmup))},
        "input_generation_s": r["gen_s"],
    }
    if not args.skip_fp64:
        k64 = min(args.steps, args.fp64_steps)
        r64 = large3d_run("f64", args.warmup + args.steps - k64, k64, tile=tile3)
        v64 = n_part * k64 / r64["wall"]
        t64 = r64["timing"]
        out["fp64"] = {"pushes_per_s": v64, "steps": k64,
                       "push_ms_per_launch": t64.ms_push / max(1, t64.n_push),
                       "note": "the same kernels instantiated in FP64, same run, timed on the last %d steps of "
                               "the same window" % k64}
        out["fp32_over_fp64"] = value / v64
        log("headline FP64: %.3e pushes/s" % v64)
    return out


def pic2d_inputs(n_cells=N_CELLS, x_min=(0.0, 0.0, -25.6), seed=2):
    """Electrons + protons of the 4096 x 1024 LG run (16 + 16 per cell),
    drawn on the GPU."""
    from paper_2307_04843_amd import inputs
    dens = inputs.density_ramp_x(0.05, 0.0, 200.0)
    dx = (LAMBDA_DX,) * 3
    e = inputs.plasma_device(2, n_cells, dx, x_min, PPC, dens, 1.0, 1.0, seed, stream=0)
    p = inputs.plasma_device(2, n_cells, dx, x_min, PPC, dens, 1.0, inputs.PROTON_MASS, seed, stream=1,
                             positions_from=e)
    return [dict(q=-1.0, m=1.0, state=e), dict(q=1.0, m=inputs.PROTON_MASS, state=p)]


INPULSE2D_CELLS = (512, 1, 1024)
INPULSE2D_XMIN = (37.0, 0.0, -25.6)


def pic2d_leg(args):
    """The 4096 x 1024 LG run (134M particles) on the last steps of its
    2000-step run (the pulse inside the ramp); then the same window in FP64,
    with the grid-sampled pulse and with the analytic current; then a box of
    512 x 1024 cells that lies inside the pulse's envelope for the whole
    window (every particle evaluates the LG pulse every step)."""
    import torch
    W2, K2 = args.warmup2d, args.steps2d
    first = window_start(RUN2_STEPS, W2, K2)

    def fresh(prec="f32", n_cells=N_CELLS, x_min=(0.0, 0.0, -25.6)):
        sp = pic2d_inputs(n_cells, x_min)
        if prec == "f64":
            for s in sp:
                for key in ("off", "u", "w"):
                    s["state"][key] = s["state"][key].to(torch.float64)
        return sp

    def summary(r, steps):
        tm = r["timing"]
        ms = tm.ms_push / max(1, tm.n_push)
        bl = r["n_part"] * 52 + r["ncell"] * 36
        return {"pushes_per_s": r["n_part"] * steps / r["wall"], "ms_per_step": r["wall"] * 1e3 / steps,
                "push_ms_per_launch": ms, "hbm_frac": bl / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "sort_ms_per_step": tm.ms_sort / steps, "yee_ms": tm.ms_yee / max(1, tm.n_yee),
                "other_ms_per_step": tm.ms_other / steps}

    out = {"workload": "2-D PIC 4096x1024 cells lambda/20, 16 e + 16 p per cell (134M), 0->0.05 n_c ramp over "
                       "200 lambda, analytic LG l=1 p=0 a0=5 w0=8 tau=30, timed steps %d..%d of the 2000-step "
                       "run" % (first + W2, first + W2 + K2), "steps": K2, "warmup": W2}
    log("2-D FP32: %d + %d steps from step %d" % (W2, K2, first))
    r = run_gpu(fresh(), "f32", K2, W2, sort_every=args.sort_every, window_shifts=12, first_step=first)
    out.update(summary(r, K2))
    out["particles"] = r["n_part"]
    out["moving_window"] = {"shift_ms": r["shift_ms"], "shift_over_step": r["shift_ms"] / out["ms_per_step"],
                            "note": "ap_shift_window on this grid between steps after the timed ones (ring "
                                    "origin moved, one column of E2, B2 cleared, the leaving column's particles "
                                    "freed, 1 e + 1 p per cell of the entering column injected into freed "
                                    "slots), wall time incl. its host synchronisation"}
    if not args.skip_fp64:
        r64 = run_gpu(fresh("f64"), "f64", K2, W2, first_step=first)
        out["fp64"] = summary(r64, K2)
        out["fp32_over_fp64"] = out["pushes_per_s"] / out["fp64"]["pushes_per_s"]
        rg = run_gpu(fresh(), "f32", K2, W2, on_grid=True, first_step=first)
        out["grid_sampled"] = summary(rg, K2)
        out["grid_sampled"]["note"] = ("E1, B1 sampled on the grid (Fig. 1 loop, AP_SAMPLE_GRID): the sampling "
                                       "kernel + the push without per-particle pulse evaluation")
        rc = run_gpu(fresh(), "f32", K2, W2, on_grid=True, current=True, first_step=first)
        out["analytic_current"] = summary(rc, K2)
        out["analytic_current"]["note"] = ("the pulse's analytic current J1 (Sec. IV, AP_DISP_PLASMA, wp2 = "
                                           "0.05, grid-sampled E1, corrected B1)")
    # every particle inside the envelope: the box spans x = 37 ... 62.6 lambda
    # and the pulse (front at v_g t, 30 lambda/c long) covers it over the window
    ri = run_gpu(fresh(n_cells=INPULSE2D_CELLS, x_min=INPULSE2D_XMIN), "f32", K2, W2, first_step=first,
                 n_cells=INPULSE2D_CELLS, x_min=INPULSE2D_XMIN)
    out["in_pulse"] = summary(ri, K2)
    out["in_pulse"]["particles"] = ri["n_part"]
    out["in_pulse"]["workload"] = ("512x1024 cells of the same run at x = 37-62.6 lambda, inside the LG "
                                   "envelope at every timed step: every push evaluates the LG pulse")
    return out


def adjoint_leg(args):
    beam = adjoint_beam()
    adj = {"workload": "gridless head-on collision: 2^24 electrons, gamma 2000 (5%% spread), "
                       "sigma_perp 1 lambda, eps^4 nonparaxial Gaussian a0=20 w0=2 tau=20, "
                       "dt=0.01, steps %d of the 20000-step run (t=%.0f..%.0f), observable "
                       "<p_perp^2>, gradient wrt (a0, w0, x_f)"
                       % (args.adj_steps, ADJ_T0, ADJ_T0 + ADJ_DT * args.adj_steps),
           "particles": ADJ_N, "steps": args.adj_steps}
    for prec in ("f32", "f64"):
        log("adjoint leg %s: %d steps" % (prec, args.adj_steps))
        adj[prec] = run_adjoint(beam, prec, args.adj_steps)
    g32, g64 = adj["f32"]["grad"], adj["f64"]["grad"]
    adj["grad_rel_diff_f32_vs_f64"] = [abs(a - b) / max(abs(b), 1e-300) for a, b in zip(g32, g64)]
    gnorm = math.sqrt(sum(b * b for b in g64))
    adj["grad_diff_over_norm_f32_vs_f64"] = [abs(a - b) / max(gnorm, 1e-300) for a, b in zip(g32, g64)]
    adj["f32_over_f64_forward"] = adj["f32"]["forward_pushes_per_s"] / adj["f64"]["forward_pushes_per_s"]
    adj["f32_over_f64_adjoint"] = adj["f32"]["adjoint_pushes_per_s"] / adj["f64"]["adjoint_pushes_per_s"]
    return adj


ADJ_FULL_STEPS = 20000   # the collision run's length (t = 0 ... 200 lambda/c)
ADJ_FULL_SLOTS = 64


def adjoint_full_leg(args):
    """The whole 20000-step collision run in FP32 (beam starting 100 lambda
    ahead of the focus, so that it meets the pulse at t = 100 lambda/c),
    differentiated with the binomial checkpoint schedule over 64 slots."""
    from paper_2307_04843_amd import apt, inputs
    steps = args.adj_full_steps
    beam = inputs.beam(ADJ_N, 2000.0, 0.05, 1.0, 1.0, 100.0, 1.0, seed=3)
    log("adjoint, whole run: %d steps, %d slots" % (steps, ADJ_FULL_SLOTS))
    r = run_adjoint(beam, "f32", steps, t0=0.0, revolve=ADJ_FULL_SLOTS)
    t, f = apt.ap_revolve_plan(steps, ADJ_FULL_SLOTS)
    r.update({"workload": "gridless head-on collision, the whole run: 2^24 electrons, gamma 2000 (5%% spread), "
                          "eps^4 nonparaxial Gaussian a0=20 w0=2 tau=20, dt=0.01, %d steps (t=0..%.0f), FP32, "
                          "gradient of <p_perp^2> wrt (a0, w0, x_f)" % (steps, steps * ADJ_DT),
              "particles": ADJ_N, "steps": steps, "revolve_repeats": t, "revolve_forward_steps": f,
              "note": "binomial checkpointing: %d whole states (%.1f GB), the recording sweep plus %d re-advanced "
                      "steps, then the reverse steps; backward_s covers re-advancing and reverse steps"
                      % (ADJ_FULL_SLOTS, r["checkpoint_gb"], f)})
    log("adjoint, whole run: forward %.1f s, backward %.1f s" % (r["forward_s"], r["backward_s"]))
    return r


def adjoint3d_long_leg(args):
    """The 512 x 256 x 256 flying-focus run's frozen-grid adjoint over a long
    window, binomial schedule over 16 whole states."""
    import torch
    from paper_2307_04843_amd import apt
    from paper_2307_04843_amd.autograd import APTRun, GriddedRun
    species = workload3d_inputs()
    n = int(species[0]["state"]["u"].shape[1])
    dt = 0.95 / math.sqrt(3) * DX3
    pp = workload3d_pulse(dt)
    steps, slots = args.adj3d_long_steps, 16
    names = ["beta_f", "chirp"]
    log("3-D adjoint, %d steps, %d slots" % (steps, slots))
    run = GriddedRun(3, N3, (DX3,) * 3, (0.0, -8.0, -8.0), species, "ff", pp, names, steps,
                     t0=T0_STEP3 * dt, dt=dt, precision="f32", revolve=slots)
    try:
        p = torch.tensor([pp["beta_f"], pp["chirp"]], dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        a = time.perf_counter()
        u, _ = APTRun.apply(p, run)
        torch.cuda.synchronize()
        b = time.perf_counter()
        obs = (u[1].double() ** 2 + u[2].double() ** 2).sum() / n
        obs.backward()
        torch.cuda.synchronize()
        c = time.perf_counter()
        t, f = apt.ap_revolve_plan(steps, slots)
        out = {"workload": "3-D PIC 512x256x256, 268M electrons, flying focus beta_f=-1 chirp 5%%, steps "
                           "%d..%d, frozen-grid adjoint of <p_perp^2> wrt (beta_f, chirp)"
                           % (T0_STEP3, T0_STEP3 + steps),
               "steps": steps, "revolve_slots": slots, "checkpoint_gb": run.ckpt.numel() / 1e9,
               "revolve_repeats": t, "revolve_forward_steps": f, "grad": p.grad.tolist(),
               "forward_s": b - a, "backward_s": c - b, "forward_pushes_per_s": n * steps / (b - a),
               "adjoint_pushes_per_s": n * steps / (c - b)}
        log("3-D adjoint: forward %.1f s, backward %.1f s" % (b - a, c - b))
        return out
    finally:
        run.close()
        del run
        torch.cuda.empty_cache()


LEGS = ("headline", "pic2d", "adjoint", "adjoint_full", "three_d", "small", "rows1d", "cpu")
OPTIONAL_LEGS = ("adjoint3d_long",)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed steps of the headline run")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps before them")
    ap.add_argument("--fp64-steps", type=int, default=50, help="timed FP64 steps (at most --steps)")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated subset of %s, or the optional %s (the headline line is always "
                         "printed)" % (",".join(LEGS), ",".join(OPTIONAL_LEGS)))
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--steps2d", type=int, default=100, help="timed steps of the 4096x1024 legs")
    ap.add_argument("--warmup2d", type=int, default=10)
    ap.add_argument("--adj-steps", type=int, default=2000)
    ap.add_argument("--adj-full-steps", type=int, default=ADJ_FULL_STEPS, help="whole-run adjoint length")
    ap.add_argument("--adj3d-long-steps", type=int, default=1000, help="optional 3-D long adjoint window")
    ap.add_argument("--sort-every", type=int, default=0, help="2-D tile re-sort interval (0: library default)")
    ap.add_argument("--steps3d", type=int, default=100, help="timed steps of the 512x256x256 leg")
    ap.add_argument("--adj3d-steps", type=int, default=32, help="adjoint window of the 3-D leg (0: none)")
    ap.add_argument("--skip-coupled", action="store_true", help="3-D leg: frozen-grid adjoint only")
    ap.add_argument("--tile3", default="", help="tile shape of the 3-D runs, e.g. 8,8,4 (default: library's)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy a device buffer of this size (a known-size kernel for "
                         "scaling HBM counters in profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one GPU only (the library has no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x]
    for x in legs:
        if x not in LEGS + OPTIONAL_LEGS:
            print("bench.py: unknown leg %r" % x, file=sys.stderr)
            sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calib_copy_mib, args.calib_copy_mib))
        del src, dst
    if "headline" in legs:
        out = headline_leg(args)
    else:
        out = {"metric": METRIC, "value": None, "unit": "pushes/s", "n_gpus": 1, "steps": 0,
               "warmup": 0, "note": "headline leg skipped (profiling run)"}
    if "pic2d" in legs:
        out["pic2d"] = pic2d_leg(args)
    if "adjoint" in legs:
        out["adjoint"] = adjoint_leg(args)
    if "adjoint_full" in legs:
        out["adjoint_full"] = adjoint_full_leg(args)
    if "adjoint3d_long" in legs:
        out["adjoint3d_long"] = adjoint3d_long_leg(args)
    if "three_d" in legs:
        out["three_d"] = three_d_leg(args)
    if "small" in legs:
        out["small"] = small_leg()
    if "rows1d" in legs:
        out["rows1d"] = rows1d_leg()
    if "cpu" in legs:
        first = window_start(RUN5_STEPS, args.warmup, args.steps) + args.warmup
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(first, args.cpu_budget)
        out["cpu_baseline_2d"] = cpu_baseline_2d()
        if "adjoint" in legs:
            log("CPU oracle baseline, gridless")
            out["cpu_baseline_gridless"] = cpu_gridless_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
