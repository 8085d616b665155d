"""Differentiable runs: torch.autograd.Function over ap_step/ap_backward.

``GridlessRun`` owns a gridless Simulation, its initial particle state and a
checkpoint buffer.  ``APTRun.apply(params, run)`` resets the particles to the
initial state, applies the pulse parameters ``params`` (float64 tensor, in the
order of ``run.param_names``, lambda units), advances ``run.n_steps`` steps with
checkpoint recording and returns the final momenta u (3, N) and the emission
proxies (N,).  Its backward calls the library's hand-written adjoint
(ap_backward) and returns dL/dparams.

``GriddedRun`` does the same for a gridded run (dim 1, 2 or 3, every species,
full loop) and one species' final momenta and proxies, ordered by particle id.
By default in the frozen-grid reading (the gradient treats the E2, B2 each
push gathered as a recorded external field); with ``coupled=True`` through
the whole loop (every species' current, the Yee update and the gather).
Without ``proxy=True`` its proxy output is identically zero.

Both store their checkpoints in segments of ``segment`` steps (default
sqrt(n_steps): memory grows with n_steps) or, with ``revolve=S``, in the
binomial schedule over S whole states (fixed memory, steps re-advanced).
"""
import math

import numpy as np
import torch

from . import apt
from .sim import Simulation

PARAM_IDS = {"a0": apt.AP_PARAM_A0, "w0": apt.AP_PARAM_W0, "x_f": apt.AP_PARAM_XF,
             "beta_f": apt.AP_PARAM_BETA_F, "chirp": apt.AP_PARAM_CHIRP}


def _set_checkpoints(run):
    if run.revolve:
        apt.ap_set_revolve(run.sim.ctx, run.ckpt.data_ptr(), run.ckpt.numel(), run.revolve)
    else:
        apt.ap_set_checkpoints(run.sim.ctx, run.ckpt.data_ptr(), run.ckpt.numel(), run.segment)


class GridlessRun:
    def __init__(self, state, pulse_kind, pulse_params, param_names, n_steps, dt, t0=0.0,
                 vcell=1.0, precision="f32", q=-1.0, m=1.0, segment=None, proxy=True, revolve=None):
        self.sim = Simulation(0, dx=(vcell,) * 3, x_min=(0.0, 0.0, 0.0), t0=t0, dt=dt, precision=precision,
                              species=[dict(q=q, m=m, state=state)], proxy=proxy)
        self.kind = pulse_kind
        self.base = dict(pulse_params)
        self.param_names = list(param_names)
        for nm in self.param_names:
            if nm not in PARAM_IDS:
                raise ValueError("unknown parameter %r" % nm)
        self.n_steps = int(n_steps)
        self.segment = int(segment or max(1, int(math.sqrt(self.n_steps))))
        self.revolve = int(revolve) if revolve else 0
        if self.revolve:
            nbytes = apt.ap_revolve_bytes(self.sim.ctx, self.revolve)
        else:
            nbytes = apt.ap_checkpoint_bytes(self.sim.ctx, self.n_steps, self.segment)
        self.ckpt = torch.empty(nbytes, dtype=torch.uint8, device=self.sim.device)
        _set_checkpoints(self)
        a = self.sim.arrays[0]
        self._init = {k: [t.clone() for t in a[k]] for k in ("icell", "off", "u")}
        self._t0 = t0

    def _reset(self):
        a = self.sim.arrays[0]
        for k in ("icell", "off", "u"):
            for dst, src in zip(a[k], self._init[k]):
                dst.copy_(src)
        if a["proxy"] is not None:
            a["proxy"].zero_()
        # rewind the clock: a fresh context keeps the library state simple
        apt.ap_destroy(self.sim.ctx)
        self.sim.ctx = apt.ap_init(self.sim.grid_desc, self.sim.sp_desc, self.sim.buffers,
                                   self.sim.stream.cuda_stream)
        _set_checkpoints(self)

    def forward(self, values):
        self._reset()
        prm = dict(self.base)
        for nm, v in zip(self.param_names, values):
            prm["x0_ff" if (nm == "x_f" and self.kind == "ff") else nm] = float(v)
        self.sim.set_pulse(self.kind, **prm)
        self.sim.step(self.n_steps, flags=apt.AP_STEP_RECORD)
        a = self.sim.arrays[0]
        u = torch.stack([t.clone() for t in a["u"]])
        if a["proxy"] is not None:
            proxy = self.sim.proxy_values(0)
        else:
            proxy = torch.zeros(u.shape[1], dtype=torch.float64, device=u.device)
        return u, proxy

    def backward(self, grad_u, grad_proxy):
        dt = self.sim.dtype
        gu = (grad_u if grad_u is not None else torch.zeros((3, self.sim.sp_desc[0].n), device=self.sim.device))
        gu = gu.to(device=self.sim.device, dtype=dt).contiguous()
        gp_ptr = None
        gp = None
        # a proxy cotangent that is zero everywhere is left out: the adjoint
        # then runs the kernel without the proxy term
        if grad_proxy is not None and grad_proxy.numel() > 0 and bool(grad_proxy.abs().max() > 0):
            gp = grad_proxy.to(device=self.sim.device, dtype=dt).contiguous()
            gp_ptr = gp.data_ptr()
        ids = [PARAM_IDS[nm] for nm in self.param_names]
        torch.cuda.synchronize(self.sim.device)
        return apt.ap_backward(self.sim.ctx, 0, gu.data_ptr(), gp_ptr, ids)

    def close(self):
        # an autograd graph may still hold this run: release its device memory now
        self.sim.close()
        self.ckpt = None
        self._init = None


class GriddedRun:
    """species: Simulation species list (plasma states with cell, off, u, w).
    fields: optional initial E2, B2 (6 arrays shaped (nz, ny, nx)), else zero.
    The gradient is of species ``species_index``'s final momenta."""

    def __init__(self, dim, n, dx, x_min, species, pulse_kind, pulse_params, param_names, n_steps, t0=0.0,
                 dt=0.0, precision="f32", fields=None, species_index=0, segment=None, tile=(0, 0, 0),
                 sort_every=0, proxy=False, coupled=False, revolve=None):
        self.sim = Simulation(dim, n=n, dx=dx, x_min=x_min, t0=t0, dt=dt, precision=precision, tile=tile,
                              sort_every=sort_every, species=species, proxy=proxy)
        self.proxy = bool(proxy)
        self.mode = apt.AP_ADJ_COUPLED if coupled else apt.AP_ADJ_FROZEN
        apt.ap_set_adjoint_mode(self.sim.ctx, self.mode)
        self.kind = pulse_kind
        self.base = dict(pulse_params)
        self.param_names = list(param_names)
        for nm in self.param_names:
            if nm not in PARAM_IDS:
                raise ValueError("unknown parameter %r" % nm)
        self.n_steps = int(n_steps)
        self.sp = int(species_index)
        self.segment = int(segment or max(1, int(math.sqrt(self.n_steps))))
        self.revolve = int(revolve) if revolve else 0
        if self.revolve:
            nbytes = apt.ap_revolve_bytes(self.sim.ctx, self.revolve)
        else:
            nbytes = apt.ap_checkpoint_bytes(self.sim.ctx, self.n_steps, self.segment)
        self.ckpt = torch.empty(nbytes, dtype=torch.uint8, device=self.sim.device)
        _set_checkpoints(self)
        self._fields = None if fields is None else [torch.as_tensor(np.asarray(f)) for f in fields]
        self._init = []
        for a in self.sim.arrays:
            self._init.append({"cell": a["cell"].clone(), "off": [t.clone() if t is not None else None
                                                                   for t in a["off"]],
                               "u": [t.clone() for t in a["u"]], "w": a["w"].clone(), "id": a["id"].clone()})

    def _reset(self):
        for a, ini in zip(self.sim.arrays, self._init):
            a["cell"].copy_(ini["cell"])
            a["w"].copy_(ini["w"])
            a["id"].copy_(ini["id"])
            for k in range(3):
                if a["off"][k] is not None:
                    a["off"][k].copy_(ini["off"][k])
                a["u"][k].copy_(ini["u"][k])
            if a["proxy"] is not None:
                a["proxy"].zero_()
        # a fresh context rewinds the clock and zeroes the grid
        apt.ap_destroy(self.sim.ctx)
        self.sim.ctx = apt.ap_init(self.sim.grid_desc, self.sim.sp_desc, self.sim.buffers,
                                   self.sim.stream.cuda_stream)
        apt.ap_set_adjoint_mode(self.sim.ctx, self.mode)
        if self._fields is not None:
            E, B, _ = self.sim.field_views()
            for k in range(3):
                E[k].copy_(self._fields[k].to(E[k].dtype))
                B[k].copy_(self._fields[3 + k].to(B[k].dtype))
        _set_checkpoints(self)

    def forward(self, values):
        self._reset()
        prm = dict(self.base)
        for nm, v in zip(self.param_names, values):
            prm["x0_ff" if (nm == "x_f" and self.kind == "ff") else nm] = float(v)
        self.sim.set_pulse(self.kind, **prm)
        self.sim.step(self.n_steps, flags=apt.AP_STEP_RECORD)
        a = self.sim.arrays[self.sp]
        u = torch.stack(a["u"])
        out = torch.empty_like(u)
        idx = a["id"].long()
        out[:, idx] = u
        proxy = torch.zeros(u.shape[1], dtype=torch.float64, device=u.device)
        if a["proxy"] is not None:
            proxy[idx] = self.sim.proxy_values(self.sp)
        return out, proxy

    def backward(self, grad_u, grad_proxy=None):
        n = self.sim.sp_desc[self.sp].n
        gu = grad_u if grad_u is not None else torch.zeros((3, n), device=self.sim.device)
        gu = gu.to(device=self.sim.device, dtype=self.sim.dtype).contiguous()
        gp = None
        if self.proxy and grad_proxy is not None and grad_proxy.numel() > 0 and bool(grad_proxy.abs().max() > 0):
            gp = grad_proxy.to(device=self.sim.device, dtype=self.sim.dtype).contiguous()   # by particle id
        ids = [PARAM_IDS[nm] for nm in self.param_names]
        torch.cuda.synchronize(self.sim.device)
        return apt.ap_backward(self.sim.ctx, self.sp, gu.data_ptr(), gp.data_ptr() if gp is not None else None, ids)

    def close(self):
        # an autograd graph may still hold this run: release its device memory now
        self.sim.close()
        self.ckpt = None
        self._init = None


class APTRun(torch.autograd.Function):
    """params (float64, CPU) -> (u_final (3, N), proxy (N,)) through the HIP path
    (``run``: a GridlessRun or a GriddedRun)."""

    @staticmethod
    def forward(ctx, params, run):
        ctx.run = run
        u, proxy = run.forward(params.detach().cpu().double().tolist())
        # the run holds one recording: a later forward replaces it
        run.generation = getattr(run, "generation", 0) + 1
        ctx.generation = run.generation
        return u, proxy

    @staticmethod
    def backward(ctx, grad_u, grad_proxy):
        if getattr(ctx.run, "generation", None) != ctx.generation:
            raise RuntimeError("APTRun: the run was forwarded again since this graph was built; its "
                               "recording (checkpoints, pulse parameters) is gone")
        g = ctx.run.backward(grad_u, grad_proxy)
        return torch.tensor(g, dtype=torch.float64), None
