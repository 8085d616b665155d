"""Device buffers for one run, allocated with torch on the caller's stream.

PyTorch is used only for device memory and the stream; every kernel comes
from libapt.so through the ap_* calls in ``apt``.
"""
import numpy as np
import torch

from . import apt


_TORCH_DTYPE = {np.dtype(np.float32): torch.float32, np.dtype(np.float64): torch.float64,
                np.dtype(np.int32): torch.int32}


def _dev(x, np_dtype, dev):
    """Device tensor of a host array (converted to np_dtype) or of a tensor
    (returned as it is when it already is a contiguous one of that type on dev)."""
    if isinstance(x, torch.Tensor):
        td = _TORCH_DTYPE[np.dtype(np_dtype)]
        if x.dtype == td and x.device == dev and x.is_contiguous():
            return x
        return x.to(device=dev, dtype=td).contiguous()
    return torch.as_tensor(np.ascontiguousarray(np.asarray(x).astype(np_dtype)), device=dev)


class Simulation:
    """One context: grid + species buffers sized by ap_query_layout.

    species: list of dicts with keys q, m and a state dict from
    ``inputs.plasma`` (cell, off, u, w) or ``inputs.beam`` (icell, off, u, w);
    the arrays may be numpy arrays or torch tensors (a device tensor of the
    working type is used in place: the run updates it).  Lengths and times in
    lambda units.  ``proxy``: every species carries an emission proxy;
    ``pulse_on_grid``: the pulse may be sampled on the grid; ``open_x`` (1-D
    rows): incoming/outgoing-wave x ends, for pulses launched through x_min
    (``set_pulse(..., sampling="boundary")``); ``moving_window``: the window
    can move along +x or -x (``shift_window``, ``step_window``); spare
    particle slots are passed as free slots (cell -1, zero weight;
    ``inputs.pad_free``).
    """

    def __init__(self, dim, n=(1, 1, 1), dx=(1.0, 1.0, 1.0), x_min=(0.0, 0.0, 0.0), t0=0.0, dt=0.0,
                 precision="f32", tile=(0, 0, 0), sort_every=0, species=(), proxy=False,
                 device="cuda:0", stream=None, pulse_on_grid=False, open_x=False, moving_window=False):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP path needs a GPU")
        apt.load()
        self.dim = dim
        self.n = tuple(int(v) for v in n)
        self.dx = tuple(float(v) for v in dx)
        self.moving_window = bool(moving_window)
        self.device = torch.device(device)
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.np_dtype = np.float64 if precision == "f64" else np.float32
        g = apt.ap_grid_desc()
        g.dim = dim
        g.precision = apt.AP_F64 if precision == "f64" else apt.AP_F32
        for a in range(3):
            g.n[a] = int(n[a])
            g.tile[a] = int(tile[a])
            g.dx[a] = float(dx[a])
            g.x_min[a] = float(x_min[a])
        g.t0 = float(t0)
        g.dt = float(dt)
        g.sort_every = int(sort_every)
        g.options = ((apt.AP_GRID_PULSE_ON_GRID if pulse_on_grid else 0)
                     | (apt.AP_GRID_PROXY if (proxy and dim > 0) else 0)
                     | (apt.AP_GRID_OPEN_X if open_x else 0)
                     | (apt.AP_GRID_MOVING_WINDOW if moving_window else 0))
        self.grid_desc = g
        self.sp_desc = []
        for sp in species:
            d = apt.ap_species_desc()
            d.q = float(sp["q"])
            d.m = float(sp["m"])
            d.n = int(sp["state"]["u"].shape[1])
            self.sp_desc.append(d)
        self.layout = apt.ap_query_layout(g, self.sp_desc)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.grid = torch.zeros(max(8, (self.layout.grid_bytes + 7) // 8 * 8), dtype=torch.uint8,
                                    device=self.device)
            self.work = torch.zeros(max(256, self.layout.work_bytes), dtype=torch.uint8,
                                    device=self.device)
        self.ncell = int(self.layout.n_cells)
        self.arrays = []
        bufs = apt.ap_buffers()
        bufs.grid = self.grid.data_ptr() if self.layout.grid_bytes else None
        bufs.work = self.work.data_ptr()
        for i, sp in enumerate(species):
            st = sp["state"]
            N = st["u"].shape[1]
            arr = {}
            dev = self.device
            if dim == 0:
                arr["icell"] = [_dev(st["icell"][a], np.int32, dev) for a in range(3)]
                arr["off"] = [_dev(st["off"][a], self.np_dtype, dev) for a in range(3)]
            else:
                arr["cell"] = _dev(st["cell"], np.int32, dev)
                act = (True, dim == 3, dim >= 2)   # 1-D rows carry an x offset only
                arr["off"] = [_dev(st["off"][a], self.np_dtype, dev) if act[a] else None for a in range(3)]
            arr["u"] = [_dev(st["u"][a], self.np_dtype, dev) for a in range(3)]
            arr["w"] = _dev(st["w"], self.np_dtype, dev)
            arr["id"] = torch.arange(N, dtype=torch.int32, device=dev)
            arr["proxy"] = (torch.zeros(2 * N, dtype=self.dtype, device=dev)
                            if proxy else None)
            p = bufs.sp[i]
            if dim == 0:
                for a in range(3):
                    p.icell[a] = arr["icell"][a].data_ptr()
            else:
                p.cell = arr["cell"].data_ptr()
            for a in range(3):
                p.off[a] = arr["off"][a].data_ptr() if arr["off"][a] is not None else None
                p.u[a] = arr["u"][a].data_ptr()
            p.w = arr["w"].data_ptr()
            p.id = arr["id"].data_ptr()
            p.proxy = arr["proxy"].data_ptr() if arr["proxy"] is not None else None
            self.arrays.append(arr)
        self.buffers = bufs
        torch.cuda.synchronize(self.device)
        self.ctx = apt.ap_init(g, self.sp_desc, bufs, self.stream.cuda_stream)

    # -- fields ------------------------------------------------------------
    def field_views(self):
        """(E, B, J) lists of 3 tensors shaped (nz, ny, nx), views of the grid block."""
        if self.dim == 0:
            raise ValueError("gridless run has no grid")
        g = self.grid.view(self.dtype)[: 9 * self.ncell].view(9, self.ncell)
        nx, ny, nz = self.grid_desc.n[0], (self.grid_desc.n[1] if self.dim == 3 else 1), self.grid_desc.n[2]
        comps = [g[k].view(nz, ny, nx) for k in range(9)]
        return comps[0:3], comps[3:6], comps[6:9]

    # -- ap_* wrappers -------------------------------------------------------
    def set_pulse(self, kind, **params):
        ptype = apt.PULSE_TYPES[kind]
        apt.ap_set_pulse(self.ctx, ptype, apt.pulse_params(**params) if ptype != apt.AP_PULSE_NONE else None)

    def shift_window(self, inject=None, direction=1):
        """Move the window one cell along +x (direction 1) or -x (-1)
        (ap_shift_window).  inject: None or, per species, None or a state dict
        (cell, off, u, w) of the new particles, cells in window columns (the
        entering column: the last for +x, the first for -x)."""
        arr = None
        keep = []
        if inject is not None:
            arr = (apt.ap_inject * len(self.sp_desc))()
            for i, st in enumerate(inject):
                if st is None or len(st["w"]) == 0:
                    continue
                cell = _dev(st["cell"], np.int32, self.device)
                off = [_dev(st["off"][k], self.np_dtype, self.device) for k in range(3)]
                u = [_dev(st["u"][k], self.np_dtype, self.device) for k in range(3)]
                w = _dev(st["w"], self.np_dtype, self.device)
                keep += [cell, w] + off + u
                arr[i].cell = cell.data_ptr()
                for k in range(3):
                    arr[i].off[k] = off[k].data_ptr() if self.arrays[i]["off"][k] is not None else None
                    arr[i].u[k] = u[k].data_ptr()
                arr[i].w = w.data_ptr()
                arr[i].n = int(w.numel())
        apt.ap_shift_window(self.ctx, direction, arr)
        del keep

    def window(self):
        """(x_min in lambda, storage origin): window column l lives in storage
        column (l + origin) mod n[0] of the fields and of the caller's cells."""
        return apt.ap_get_window(self.ctx)

    def window_due(self, beta, x_ref, t_ref):
        return apt.ap_window_due(self.ctx, beta, x_ref, t_ref)

    def step_window(self, n, beta, x_ref, t_ref, inject=None):
        """n steps with the window following x_ref + beta (t - t_ref): before
        each step, shift while a shift is due.  inject(direction, x_min_new):
        None or the per-species injection of the entering column."""
        shifts = 0
        for _ in range(n):
            while True:
                d = self.window_due(beta, x_ref, t_ref)
                if d == 0:
                    break
                x_new = self.window()[0] + d * self.dx[0]
                self.shift_window(inject(d, x_new) if inject is not None else None, d)
                shifts += d
            self.step(1)
        return shifts

    def window_fields(self):
        """Copies of E2, B2 in window column order (ring origin undone)."""
        E, B, _ = self.field_views()
        o = self.window()[1]
        return [torch.roll(f, -o, dims=2).clone() for f in E], [torch.roll(f, -o, dims=2).clone() for f in B]

    def eval_pulse(self, xyz, t):
        """E1, B1 at lab points xyz (3, n) in lambda units, time t; numpy (3, n) arrays."""
        pts = torch.as_tensor(np.ascontiguousarray(xyz, dtype=np.float64), device=self.device)
        n = pts.shape[1]
        E = torch.empty(3 * n, dtype=self.dtype, device=self.device)
        B = torch.empty(3 * n, dtype=self.dtype, device=self.device)
        apt.ap_eval_pulse(self.ctx, n, pts.data_ptr(), t, E.data_ptr(), B.data_ptr())
        torch.cuda.synchronize(self.device)
        return E.view(3, n).double().cpu().numpy(), B.view(3, n).double().cpu().numpy()

    def step(self, n=1, flags=0):
        apt.ap_step(self.ctx, n, flags)

    def diag(self, what=apt.AP_DIAG_PARTICLES | apt.AP_DIAG_FIELDS, allow_numeric=False):
        return apt.ap_gather_diag(self.ctx, what, allow_numeric=allow_numeric)

    def time(self):
        return apt.ap_get_time(self.ctx)

    def state(self, i):
        """Host copy of species i, ordered by particle id."""
        torch.cuda.synchronize(self.device)
        a = self.arrays[i]
        ids = a["id"].cpu().numpy()
        order = np.argsort(ids, kind="stable")
        out = {"id": ids[order]}
        if self.dim == 0:
            out["icell"] = np.stack([a["icell"][k].cpu().numpy()[order] for k in range(3)])
            out["off"] = np.stack([a["off"][k].cpu().numpy()[order] for k in range(3)])
        else:
            cell = a["cell"].cpu().numpy()[order]
            if self.moving_window:
                # storage cells -> window cells (free slots keep -1)
                o = self.window()[1]
                nx = self.n[0]
                col = cell % nx
                cell = np.where(cell >= 0, cell - col + (col - o) % nx, cell)
            out["cell"] = cell
            out["off"] = np.stack([a["off"][k].cpu().numpy()[order] if a["off"][k] is not None
                                   else np.zeros(len(ids), dtype=self.np_dtype) for k in range(3)])
        out["u"] = np.stack([a["u"][k].cpu().numpy()[order] for k in range(3)])
        out["w"] = a["w"].cpu().numpy()[order]
        if a["proxy"] is not None:
            out["proxy"] = self.proxy_values(i).cpu().numpy()[order]
        return out

    def proxy_values(self, i):
        """Per-particle emission proxies of species i (FP64 device tensor, slot
        order), read out by the library (ap_read_proxy)."""
        n = self.sp_desc[i].n
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        apt.ap_read_proxy(self.ctx, i, out.data_ptr())
        torch.cuda.synchronize(self.device)
        return out

    def close(self):
        """Destroy the context and drop the device buffers (state() and the
        field views are unavailable afterwards)."""
        if getattr(self, "ctx", None):
            torch.cuda.synchronize(self.device)
            apt.ap_destroy(self.ctx)
            self.ctx = None
            self.grid = self.work = None
            self.arrays = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
