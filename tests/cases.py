"""Seeded cases shared by the parity tests: one input, two consumers.

``make_case`` draws a plasma (and optional random internal fields) from the
shared input generator and returns it together with the lambda-unit run
description; ``oracle_state`` turns it into oracle objects, and the HIP side
uploads the same arrays through ``paper_2307_04843_amd.sim``.
"""
import math

import numpy as np

from oracle import pic, pulses, units
from paper_2307_04843_amd import inputs

L = units.LAMBDA


def cfg2_pulse(dx, dt):
    """Laguerre-Gaussian l=1, p=0 pulse of the 4096x1024 ramp workload (lambda units):
    a0 = 5 (peak), w0 = 8, tau = 30, focus at the box centre, front at x = 0 at t = 0."""
    x_f = 102.4
    tau = 30.0
    vg = units.dispersion(units.DISP_PAPER2, dx * L, dt * L)[1]
    return dict(type="lg", a0=5.0, tau=tau, x_ref=x_f, t_ref=tau / 2 + x_f / vg, x_f=x_f, w0=8.0,
                y_c=0.0, z_c=0.0, q_slice=0.0, d_f=3, lg_l=1, lg_p=0, pol=1,
                dispersion=units.DISP_PAPER2, dx_prop=dx, dt_prop=dt, dt=dt)


def cfg1_pulse(dx, dt, nx=128, nz=64):
    """Paraxial Gaussian of the 128x64 2-D workload: a0 = 1, w0 = 5, tau = 10,
    focus at the box centre, front at x_min at t = 0 (lambda units)."""
    x_f = nx * dx / 2
    z_c = nz * dx / 2
    tau = 10.0
    vg = units.dispersion(units.DISP_PAPER2, dx * L, dt * L)[1]
    return dict(type="gauss", a0=1.0, tau=tau, x_ref=x_f, t_ref=tau / 2 + x_f / vg, x_f=x_f, w0=5.0,
                z_c=z_c, d_f=2, pol=1, dispersion=units.DISP_PAPER2, dx_prop=dx, dt_prop=dt, dt=dt)


def make_case(dim=2, n=(70, 1, 40), dxl=0.05, x_min=(48.0, 0.0, 4.8), t0_steps=1900, ppc=4,
              species=("e", "p"), pulse="cfg2", field_amp=0.05, u_scale=1.0, seed=1):
    """A small replica placed where the pulse is present; returns a dict."""
    dx = (dxl, dxl, dxl)
    dt = units.default_dt(dxl, dim)   # c dt/dx = 0.95/sqrt(D), lambda units
    t0 = t0_steps * dt
    sp = []
    base = None
    for s_i, kind in enumerate(species):
        m = 1.0 if kind == "e" else inputs.PROTON_MASS
        q = -1.0 if kind == "e" else 1.0
        st = inputs.plasma(dim, n, dx, x_min, ppc, inputs.density_uniform(0.05), 1.0, m, seed,
                           stream=s_i, positions_from=base)
        if u_scale != 1.0:
            st["u"] = (st["u"] * np.float32(u_scale)).astype(np.float32)
        if base is None:
            base = st
        sp.append(dict(q=q, m=m, state=st))
    rng = np.random.Generator(np.random.Philox(key=seed + 77))
    shape = (n[2], n[1] if dim == 3 else 1, n[0])
    fields = [(rng.standard_normal(shape) * field_amp).astype(np.float32) for _ in range(6)]
    if pulse == "cfg2":
        pp = cfg2_pulse(dxl, dt)
    elif pulse == "cfg1":
        pp = cfg1_pulse(dxl, dt)
    elif pulse is None:
        pp = None
    else:
        pp = pulse
    return dict(dim=dim, n=n, dx=dx, x_min=x_min, t0=t0, dt=dt, species=sp, fields=fields, pulse=pp)


def oracle_state(case, proxy=False):
    """Oracle Grid, Species list and Pulse for a case (internal units); with
    ``proxy`` every species accumulates the emission proxy from zero."""
    dim = case["dim"]
    n = case["n"]
    g = pic.Grid(dim, n, tuple(d * L for d in case["dx"]), case["dt"] * L,
                 tuple(v * L for v in case["x_min"]), t0=case["t0"] * L)
    for k in range(3):
        g.E[k][...] = case["fields"][k].astype(float)
        g.B[k][...] = case["fields"][3 + k].astype(float)
    sps = []
    for sp in case["species"]:
        st = sp["state"]
        nx, ny = n[0], (n[1] if dim == 3 else 1)
        cell = st["cell"].astype(np.int64)
        pos = np.zeros((3, cell.size))
        pos[0] = (cell % nx) + st["off"][0].astype(float)
        if dim == 3:
            pos[1] = ((cell // nx) % ny) + st["off"][1].astype(float)
        pos[2] = (cell // (nx * ny)) + st["off"][2].astype(float)
        sps.append(pic.Species(sp["q"], sp["m"], pos, st["u"].astype(float), st["w"].astype(float),
                               proxy=np.zeros(cell.size) if proxy else None))
    P = pulses.Pulse(case["pulse"]) if case["pulse"] is not None else None
    return g, sps, P


def gpu_positions(case, st):
    """Cell-unit positions (3, N) from a GPU state dict."""
    dim = case["dim"]
    n = case["n"]
    nx, ny = n[0], (n[1] if dim == 3 else 1)
    cell = st["cell"].astype(np.int64)
    pos = np.zeros((3, cell.size))
    pos[0] = (cell % nx) + st["off"][0].astype(float)
    if dim == 3:
        pos[1] = ((cell // nx) % ny) + st["off"][1].astype(float)
    pos[2] = (cell // (nx * ny)) + st["off"][2].astype(float)
    return pos


def periodic_diff(a, b, n):
    d = a - b
    return d - n * np.round(d / n)


def sim_from_case(case, precision="f32", tile=(0, 0, 0), sort_every=0, pulse_on_grid=False, proxy=False,
                  moving_window=False):
    from paper_2307_04843_amd.sim import Simulation
    sim = Simulation(case["dim"], n=case["n"], dx=case["dx"], x_min=case["x_min"], t0=case["t0"],
                     dt=case["dt"], precision=precision, tile=tile, sort_every=sort_every,
                     species=case["species"], pulse_on_grid=pulse_on_grid, proxy=proxy,
                     moving_window=moving_window)
    E, B, _ = sim.field_views()
    import torch
    for k in range(3):
        E[k].copy_(torch.as_tensor(case["fields"][k]).to(E[k].dtype))
        B[k].copy_(torch.as_tensor(case["fields"][3 + k]).to(B[k].dtype))
    if case["pulse"] is not None:
        pp = {k: v for k, v in case["pulse"].items() if k not in ("type", "dt")}
        if pulse_on_grid:
            pp["sampling"] = "grid"
        sim.set_pulse(case["pulse"]["type"], **pp)
    else:
        sim.set_pulse("none")
    return sim


def force_scale(g, sps, P):
    """|q/m| dt (|E_tot| + |Gamma F|) per particle at the step's start (oracle fields).

    The local laser amplitude |Gamma F| enters because the carrier phase is
    only defined to the precision of its FP64 terms (~1e-13 rad at 10^3 rad):
    at a zero crossing of the carrier the instantaneous field is small but its
    rounding error is set by the amplitude."""
    out = []
    for sp in sps:
        E2, _ = pic.gather(g, sp.pos)
        X, Y, Z = pic.lab_positions(g, sp.pos, P.q_slice)
        E1, _ = pulses.analytic_fields(P, g.t, X, Y, Z)
        amp = pulses._envelope(P, g.t, X)[0] * np.abs(pulses._profile(P, g.t, X, Y, Z)[0])
        out.append(abs(sp.q / sp.m) * g.dt * (np.linalg.norm(E1 + E2, axis=0) + amp))
    return out
