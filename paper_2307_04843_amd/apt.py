"""Thin ctypes binding of libapt.so (the C ABI in include/apt.h).

Functions keep the C names (ap_query_layout, ap_init, ap_set_pulse, ap_step,
ap_gather_diag, ap_backward, ap_destroy, ...) and only marshal arguments;
every step of the method runs in the HIP kernels of the library.  The
library must be built (``python -m paper_2307_04843_amd.build``): importing
this module without it raises, there is no fallback.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapt.so")

AP_OK, AP_E_ARG, AP_E_STATE, AP_E_DEVICE, AP_E_NOMEM, AP_E_UNSUPPORTED, AP_E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
AP_MAX_SPECIES = 4
AP_F32, AP_F64 = 0, 1
AP_PULSE_NONE, AP_PULSE_PLANE, AP_PULSE_GAUSS, AP_PULSE_LG, AP_PULSE_FF, AP_PULSE_GAUSS_NP = range(6)
AP_DISP_PAPER2, AP_DISP_EXACT, AP_DISP_VACUUM, AP_DISP_PLASMA = 0, 1, 2, 3
AP_STEP_CONTINUITY, AP_STEP_NO_YEE, AP_STEP_RECORD = 0x1, 0x2, 0x4
AP_DIAG_PARTICLES, AP_DIAG_FIELDS = 0x1, 0x2
AP_PARAM_A0, AP_PARAM_W0, AP_PARAM_XF, AP_PARAM_BETA_F, AP_PARAM_CHIRP = range(5)
AP_GRID_PULSE_ON_GRID = 0x1
AP_GRID_PROXY = 0x2
AP_GRID_OPEN_X = 0x4
AP_GRID_MOVING_WINDOW = 0x8
AP_ADJ_FROZEN, AP_ADJ_COUPLED = 0, 1
AP_ENV_SIN2, AP_ENV_SGAUSS = 0, 1
AP_SAMPLE_PARTICLES, AP_SAMPLE_GRID, AP_SAMPLE_BOUNDARY = 0, 1, 2
ENVELOPES = {"sin2": AP_ENV_SIN2, "sgauss": AP_ENV_SGAUSS}
SAMPLINGS = {"particles": AP_SAMPLE_PARTICLES, "grid": AP_SAMPLE_GRID, "boundary": AP_SAMPLE_BOUNDARY}

PULSE_TYPES = {"none": AP_PULSE_NONE, "plane": AP_PULSE_PLANE, "gauss": AP_PULSE_GAUSS,
               "lg": AP_PULSE_LG, "ff": AP_PULSE_FF, "gauss_np": AP_PULSE_GAUSS_NP}

EXPORTED = ("ap_query_layout", "ap_init", "ap_set_pulse", "ap_step", "ap_gather_diag", "ap_gather_diag_static",
            "ap_get_time", "ap_eval_pulse", "ap_read_proxy", "ap_set_checkpoints", "ap_set_adjoint_mode",
            "ap_checkpoint_bytes", "ap_backward", "ap_timing_enable", "ap_timing_read", "ap_shift_window",
            "ap_get_window", "ap_window_due", "ap_set_revolve", "ap_revolve_bytes", "ap_revolve_plan",
            "ap_destroy", "ap_last_error")


class ap_grid_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("n", C.c_int32 * 3),
                ("tile", C.c_int32 * 3), ("dx", C.c_double * 3), ("x_min", C.c_double * 3),
                ("t0", C.c_double), ("dt", C.c_double), ("sort_every", C.c_int32),
                ("options", C.c_int32)]


class ap_species_desc(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("n", C.c_int64)]


class ap_particles(C.Structure):
    _fields_ = [("cell", C.c_void_p), ("icell", C.c_void_p * 3), ("off", C.c_void_p * 3),
                ("u", C.c_void_p * 3), ("w", C.c_void_p), ("id", C.c_void_p), ("proxy", C.c_void_p)]


class ap_inject(C.Structure):
    _fields_ = [("cell", C.c_void_p), ("off", C.c_void_p * 3), ("u", C.c_void_p * 3), ("w", C.c_void_p),
                ("n", C.c_int64)]


class ap_layout(C.Structure):
    _fields_ = [("grid_bytes", C.c_size_t), ("work_bytes", C.c_size_t), ("real_bytes", C.c_size_t),
                ("n_cells", C.c_int64), ("n_tiles", C.c_int64), ("ckpt_slot_bytes", C.c_size_t)]


class ap_buffers(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("work", C.c_void_p), ("sp", ap_particles * AP_MAX_SPECIES)]


class ap_pulse_params(C.Structure):
    _fields_ = [("a0", C.c_double), ("tau", C.c_double), ("t_ref", C.c_double), ("x_ref", C.c_double),
                ("phi0", C.c_double), ("chirp", C.c_double), ("x_f", C.c_double), ("w0", C.c_double),
                ("y_c", C.c_double), ("z_c", C.c_double), ("q_slice", C.c_double),
                ("beta_f", C.c_double), ("x0_ff", C.c_double), ("t0_ff", C.c_double),
                ("dx_prop", C.c_double), ("dt_prop", C.c_double),
                ("d_f", C.c_int32), ("lg_l", C.c_int32), ("lg_p", C.c_int32), ("pol", C.c_int32),
                ("dispersion", C.c_int32), ("np_order", C.c_int32),
                ("envelope", C.c_int32), ("sg_order", C.c_int32), ("sampling", C.c_int32),
                ("no_fd", C.c_int32), ("fwhm", C.c_double), ("wp2", C.c_double), ("zeta", C.c_double)]


class ap_diag(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int64), ("field_energy", C.c_double),
                ("sum_w", C.c_double * 4), ("kinetic", C.c_double * 4),
                ("mean_u", (C.c_double * 3) * 4), ("mean_u2", (C.c_double * 3) * 4),
                ("mean_gamma", C.c_double * 4), ("proxy_sum", C.c_double * 4),
                ("continuity_max", C.c_double), ("j_max", C.c_double),
                ("n_nonfinite", C.c_int64), ("n_fast", C.c_int64),
                ("n_offtile", C.c_int64), ("n_skipped", C.c_int64)]


class ap_timing(C.Structure):
    _fields_ = [("ms_push", C.c_double), ("ms_yee", C.c_double), ("ms_sort", C.c_double),
                ("ms_other", C.c_double), ("n_push", C.c_int64), ("n_yee", C.c_int64),
                ("n_sort", C.c_int64), ("n_other", C.c_int64), ("pushes", C.c_int64)]


class APTError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__("%s failed with status %d: %s" % (where, status, msg))
        self.status = status


_lib = None


def load():
    """Load libapt.so from the package directory (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libapt.so is not built: run `python -m paper_2307_04843_amd.build` "
                          "(the HIP path has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    sig = {
        "ap_query_layout": (C.c_int32, [P(ap_grid_desc), P(ap_species_desc), C.c_int32, P(ap_layout)]),
        "ap_init": (C.c_int32, [P(ap_grid_desc), P(ap_species_desc), C.c_int32, P(ap_buffers),
                                C.c_void_p, P(C.c_void_p)]),
        "ap_set_pulse": (C.c_int32, [C.c_void_p, C.c_int32, P(ap_pulse_params)]),
        "ap_step": (C.c_int32, [C.c_void_p, C.c_int64, C.c_uint32]),
        "ap_gather_diag": (C.c_int32, [C.c_void_p, C.c_uint32, P(ap_diag)]),
        "ap_gather_diag_static": (C.c_int32, [C.c_void_p, C.c_uint32, P(ap_diag)]),
        "ap_get_time": (C.c_int32, [C.c_void_p, P(C.c_double), P(C.c_int64)]),
        "ap_eval_pulse": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_double, C.c_void_p,
                                      C.c_void_p]),
        "ap_read_proxy": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
        "ap_set_checkpoints": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32]),
        "ap_checkpoint_bytes": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int32, P(C.c_size_t)]),
        "ap_set_revolve": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32]),
        "ap_revolve_bytes": (C.c_int32, [C.c_void_p, C.c_int32, P(C.c_size_t)]),
        "ap_revolve_plan": (C.c_int32, [C.c_int64, C.c_int32, P(C.c_int64), P(C.c_int64)]),
        "ap_set_adjoint_mode": (C.c_int32, [C.c_void_p, C.c_int32]),
        "ap_backward": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, P(C.c_int32),
                                    C.c_int32, P(C.c_double)]),
        "ap_timing_enable": (C.c_int32, [C.c_void_p, C.c_int32]),
        "ap_timing_read": (C.c_int32, [C.c_void_p, P(ap_timing), C.c_int32]),
        "ap_shift_window": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
        "ap_get_window": (C.c_int32, [C.c_void_p, P(C.c_double), P(C.c_int32)]),
        "ap_window_due": (C.c_int32, [C.c_void_p, C.c_double, C.c_double, C.c_double, P(C.c_int32)]),
        "ap_destroy": (C.c_int32, [C.c_void_p]),
        "ap_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error():
    return load().ap_last_error().decode()


def _check(status, where, allow=()):
    if status != AP_OK and status not in allow:
        raise APTError(status, where, last_error())
    return status


def ap_query_layout(grid, species):
    lib = load()
    arr = (ap_species_desc * len(species))(*species)
    out = ap_layout()
    _check(lib.ap_query_layout(C.byref(grid), arr, len(species), C.byref(out)), "ap_query_layout")
    return out


def ap_init(grid, species, buffers, stream_ptr):
    lib = load()
    arr = (ap_species_desc * len(species))(*species)
    ctx = C.c_void_p()
    _check(lib.ap_init(C.byref(grid), arr, len(species), C.byref(buffers), C.c_void_p(stream_ptr),
                       C.byref(ctx)), "ap_init")
    return ctx


def ap_set_pulse(ctx, pulse_type, params):
    _check(load().ap_set_pulse(ctx, pulse_type, C.byref(params) if params is not None else None),
           "ap_set_pulse")


def ap_step(ctx, n_steps, flags=0):
    _check(load().ap_step(ctx, int(n_steps), int(flags)), "ap_step")


def ap_gather_diag(ctx, what=AP_DIAG_PARTICLES | AP_DIAG_FIELDS, allow_numeric=False):
    out = ap_diag()
    st = load().ap_gather_diag(ctx, int(what), C.byref(out))
    _check(st, "ap_gather_diag", allow=(AP_E_NUMERIC,) if allow_numeric else ())
    return out, st


def ap_gather_diag_static(ctx, what=AP_DIAG_PARTICLES | AP_DIAG_FIELDS, allow_numeric=False):
    out = ap_diag()
    st = load().ap_gather_diag_static(ctx, int(what), C.byref(out))
    _check(st, "ap_gather_diag_static", allow=(AP_E_NUMERIC,) if allow_numeric else ())
    return out, st


def ap_get_time(ctx):
    t = C.c_double()
    s = C.c_int64()
    _check(load().ap_get_time(ctx, C.byref(t), C.byref(s)), "ap_get_time")
    return t.value, s.value


def ap_eval_pulse(ctx, n, xyz_ptr, t, e_ptr, b_ptr):
    _check(load().ap_eval_pulse(ctx, int(n), C.c_void_p(xyz_ptr), float(t), C.c_void_p(e_ptr),
                                C.c_void_p(b_ptr)), "ap_eval_pulse")


def ap_read_proxy(ctx, species, dst_ptr):
    _check(load().ap_read_proxy(ctx, int(species), C.c_void_p(dst_ptr)), "ap_read_proxy")


def ap_set_checkpoints(ctx, dev_ptr, nbytes, segment):
    _check(load().ap_set_checkpoints(ctx, C.c_void_p(dev_ptr), int(nbytes), int(segment)),
           "ap_set_checkpoints")


def ap_set_adjoint_mode(ctx, mode):
    _check(load().ap_set_adjoint_mode(ctx, int(mode)), "ap_set_adjoint_mode")


def ap_checkpoint_bytes(ctx, n_steps, segment):
    out = C.c_size_t(0)
    _check(load().ap_checkpoint_bytes(ctx, int(n_steps), int(segment), C.byref(out)), "ap_checkpoint_bytes")
    return int(out.value)


def ap_set_revolve(ctx, dev_ptr, nbytes, slots):
    _check(load().ap_set_revolve(ctx, C.c_void_p(dev_ptr), int(nbytes), int(slots)), "ap_set_revolve")


def ap_revolve_bytes(ctx, slots):
    out = C.c_size_t(0)
    _check(load().ap_revolve_bytes(ctx, int(slots), C.byref(out)), "ap_revolve_bytes")
    return int(out.value)


def ap_revolve_plan(n_steps, slots):
    """(repetitions t, forward steps of the reverse sweep) of the binomial schedule."""
    t = C.c_int64(0)
    f = C.c_int64(0)
    _check(load().ap_revolve_plan(int(n_steps), int(slots), C.byref(t), C.byref(f)), "ap_revolve_plan")
    return int(t.value), int(f.value)


def ap_backward(ctx, species, dl_du_ptr, dl_dproxy_ptr, param_ids):
    n = len(param_ids)
    ids = (C.c_int32 * n)(*param_ids)
    out = (C.c_double * n)()
    _check(load().ap_backward(ctx, int(species), C.c_void_p(dl_du_ptr), C.c_void_p(dl_dproxy_ptr or 0),
                              ids, n, out), "ap_backward")
    return list(out)


def ap_timing_enable(ctx, enable=True):
    _check(load().ap_timing_enable(ctx, 1 if enable else 0), "ap_timing_enable")


def ap_timing_read(ctx, reset=False):
    out = ap_timing()
    _check(load().ap_timing_read(ctx, C.byref(out), 1 if reset else 0), "ap_timing_read")
    return out


def ap_shift_window(ctx, direction, inject):
    """direction: +1 or -1; inject: None or a ctypes array of ap_inject, one per species."""
    _check(load().ap_shift_window(ctx, int(direction), C.cast(inject, C.c_void_p) if inject is not None else None),
           "ap_shift_window")


def ap_get_window(ctx):
    """(x_min in lambda, storage origin) of the moving window."""
    x = C.c_double()
    o = C.c_int32()
    _check(load().ap_get_window(ctx, C.byref(x), C.byref(o)), "ap_get_window")
    return x.value, o.value


def ap_window_due(ctx, beta, x_ref, t_ref):
    """+1 / -1 when the window lags x_ref + beta (t - t_ref) by half a cell or more, else 0."""
    d = C.c_int32()
    _check(load().ap_window_due(ctx, float(beta), float(x_ref), float(t_ref), C.byref(d)), "ap_window_due")
    return d.value


def ap_destroy(ctx):
    if ctx:
        _check(load().ap_destroy(ctx), "ap_destroy")


def pulse_params(**kw):
    """ap_pulse_params from keyword arguments (lambda units); defaults as in apt.h."""
    p = ap_pulse_params()
    defaults = dict(a0=1.0, tau=10.0, t_ref=0.0, x_ref=0.0, phi0=0.0, chirp=0.0, x_f=0.0, w0=5.0,
                    y_c=0.0, z_c=0.0, q_slice=0.0, beta_f=0.0, x0_ff=0.0, t0_ff=0.0, dx_prop=0.0,
                    dt_prop=0.0, d_f=3, lg_l=0, lg_p=0, pol=0, dispersion=AP_DISP_PAPER2, np_order=4,
                    envelope=AP_ENV_SIN2, sg_order=4, sampling=AP_SAMPLE_PARTICLES, fwhm=0.0, wp2=0.0,
                    zeta=0.0, no_fd=0)
    if "fd" in kw:
        kw = dict(kw)
        kw["no_fd"] = 0 if kw.pop("fd") else 1
    defaults.update(kw)
    if isinstance(defaults["envelope"], str):
        defaults["envelope"] = ENVELOPES[defaults["envelope"]]
    if isinstance(defaults["sampling"], str):
        defaults["sampling"] = SAMPLINGS[defaults["sampling"]]
    for k, v in defaults.items():
        setattr(p, k, v)
    return p
