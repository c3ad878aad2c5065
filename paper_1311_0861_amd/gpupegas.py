"""Thin ctypes binding of libgpupegas.so (include/gpupegas.h).

Argument marshalling only: every step of the timestep runs in the library's
HIP kernels.  Functions keep the C names; ``Sim`` is a small convenience
wrapper over them.  If the library is missing this module raises at import:
there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpupegas.so")

GP_OK, GP_E_INVALID, GP_E_NOMEM, GP_E_HIP, GP_E_NONFINITE, GP_E_NONPOSITIVE, GP_E_UNSUPPORTED, GP_E_STATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
GP_BC_OUTFLOW, GP_BC_PERIODIC = 0, 1
GP_FP64, GP_FP32 = 0, 1
GP_POISSON_PERIODIC, GP_POISSON_ISOLATED = 0, 1
GP_STAGE_EUL, GP_STAGE_LAG, GP_STAGE_POISSON, GP_STAGE_FINALIZE = 0, 1, 2, 3
FIELD_NAMES = [
    "rho", "mx", "my", "mz", "E", "e",
    "n", "qx", "qy", "qz",
    "Pxx", "Pxy", "Pxz", "Pyy", "Pyz", "Pzz",
    "Wxx", "Wxy", "Wxz", "Wyy", "Wyz", "Wzz",
]
GP_PHI = 22
KERNEL_NAMES = ["eul_gas", "eul_bme", "lag_gas", "lag_bme", "fft_xy_fwd", "fft_z_green", "fft_xy_inv", "finalize"]
GP_FFT_AUTO, GP_FFT_LINES = 0, 1  # x and y transforms: per half z plane where it fits, or separate passes
CELL_KERNELS = ["eul_gas", "eul_bme", "lag_gas", "lag_bme"]  # persistent, launch size settable


class gp_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("G", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("fixed_dt", ctypes.c_double),
        ("t_end", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("poisson", ctypes.c_int32),
        ("cool_lambda", ctypes.c_double),
        ("cool_alpha", ctypes.c_double),
        ("cool_theta_min", ctypes.c_double),
        ("gext", ctypes.c_double * 3),
    ]


class gp_diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("t", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("mass_gas", ctypes.c_double),
        ("mass_bme", ctypes.c_double),
        ("mom", ctypes.c_double * 3),
        ("e_gas", ctypes.c_double),
        ("e_bme", ctypes.c_double),
        ("e_pot", ctypes.c_double),
        ("kappa_gas", ctypes.c_double),
        ("kappa_bme", ctypes.c_double),
        ("outflow_gas", ctypes.c_double),
        ("outflow_bme", ctypes.c_double),
        ("n_sync_gas", ctypes.c_double),
        ("n_sync_bme", ctypes.c_double),
        ("err", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
    ]


class GpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("gpupegas status %d: %s" % (status, msg))
        self.status = status


def _load():
    # PyTorch ships its own HIP runtime under the same soname as ROCm's but
    # asks for it by another file name.  Loaded first, it satisfies the
    # library's dependency too, so the process holds one runtime; loaded
    # after the library it would bring a second one, which then sees no
    # device for the other.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgpupegas.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "gp_create": ([ctypes.POINTER(gp_config), vp, ctypes.POINTER(vp)], i32),
        "gp_destroy": ([vp], i32),
        "gp_set_field": ([vp, i32, vp, i32, i32], i32),
        "gp_get_field": ([vp, i32, vp, i32, i32], i32),
        "gp_get_potential": ([vp, vp, i32, i32], i32),
        "gp_step": ([vp, i32], i32),
        "gp_sync": ([vp], i32),
        "gp_get_diag": ([vp, ctypes.POINTER(gp_diag), i32, ctypes.POINTER(i32)], i32),
        "gp_set_time": ([vp, dbl, i64], i32),
        "gp_get_time": ([vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(i64)], i32),
        "gp_debug_stage": ([vp, i32], i32),
        "gp_time_kernels": ([vp, i32, ctypes.POINTER(dbl), i32], i32),
        "gp_use_graph": ([vp, i32], i32),
        "gp_status_str": ([i32], ctypes.c_char_p),
        "gp_last_error": ([vp], ctypes.c_char_p),
        "gp_algorithmic_bytes_per_cell": ([vp, i32], dbl),
        "gp_set_launch": ([vp, i32, i32], i32),
        "gp_get_launch": ([vp, i32, ctypes.POINTER(i32)], i32),
        "gp_set_fft_form": ([vp, i32], i32),
        "gp_set_tiling": ([vp, i32, i32, i32], i32),
        "gp_get_tiling": ([vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "gp_batch_set_tiling": ([vp, i32, i32, i32], i32),
        "gp_batch_get_tiling": ([vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "gp_batch_create": ([ctypes.POINTER(gp_config), i32, vp, ctypes.POINTER(vp)], i32),
        "gp_batch_destroy": ([vp], i32),
        "gp_batch_set_field": ([vp, i32, i32, vp, i32, i32], i32),
        "gp_batch_get_field": ([vp, i32, i32, vp, i32, i32], i32),
        "gp_batch_get_potential": ([vp, i32, vp, i32, i32], i32),
        "gp_batch_step": ([vp, i32], i32),
        "gp_batch_sync": ([vp], i32),
        "gp_batch_get_diag": ([vp, i32, ctypes.POINTER(gp_diag), i32, ctypes.POINTER(i32)], i32),
        "gp_batch_time_kernels": ([vp, i32, ctypes.POINTER(dbl), i32], i32),
        "gp_batch_set_launch": ([vp, i32, i32], i32),
        "gp_batch_get_launch": ([vp, i32, ctypes.POINTER(i32)], i32),
        "gp_batch_set_fft_form": ([vp, i32], i32),
        "gp_batch_algorithmic_bytes_per_cell": ([vp, i32], dbl),
        "gp_batch_cells": ([vp], i64),
        "gp_batch_last_error": ([vp], ctypes.c_char_p),
        "gp_potential_noalloc": ([ctypes.POINTER(gp_config), vp, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def _check(sim, status, batch=False, create=False):
    if status != GP_OK:
        detail = ""
        if sim:
            detail = (lib.gp_batch_last_error(sim) if batch else lib.gp_last_error(sim)).decode()
        elif create:
            detail = lib.gp_last_error(None).decode()
        raise GpError(status, lib.gp_status_str(status).decode() + (" (" + detail + ")" if detail else ""))


def make_config(cfg):
    """gp_config from the workload dict (keys n, lo, hi, gamma, G, cfl, eta,
    fixed_dt, t_end, bc, precision, poisson, cool_lambda, cool_alpha,
    cool_theta_min, gext)."""
    c = gp_config()
    for d in range(3):
        c.n[d] = int(cfg["n"][d])
        c.bc[d] = int(cfg.get("bc", (0, 0, 0))[d])
        c.lo[d] = float(cfg.get("lo", (-1.0,) * 3)[d])
        c.hi[d] = float(cfg.get("hi", (1.0,) * 3)[d])
    c.gamma = float(cfg.get("gamma", 5.0 / 3.0))
    c.G = float(cfg.get("G", 1.0))
    c.cfl = float(cfg.get("cfl", 0.2))
    c.eta = float(cfg.get("eta", 1e-3))
    c.fixed_dt = float(cfg.get("fixed_dt", 0.0))
    c.t_end = float(cfg.get("t_end", 0.0))
    prec = cfg.get("precision", "fp64")
    c.precision = GP_FP32 if prec in ("fp32", GP_FP32) else GP_FP64
    pois = cfg.get("poisson", "periodic")
    c.poisson = {"periodic": GP_POISSON_PERIODIC, "isolated": GP_POISSON_ISOLATED}.get(pois, pois)
    c.cool_lambda = float(cfg.get("cool_lambda", 0.0))
    c.cool_alpha = float(cfg.get("cool_alpha", 0.0))
    c.cool_theta_min = float(cfg.get("cool_theta_min", 0.0))
    for d in range(3):
        c.gext[d] = float(cfg.get("gext", (0.0, 0.0, 0.0))[d])
    return c


def gp_create(cfg, stream=None):
    c = cfg if isinstance(cfg, gp_config) else make_config(cfg)
    h = ctypes.c_void_p()
    _check(None, lib.gp_create(ctypes.byref(c), stream, ctypes.byref(h)), create=True)
    return h


def gp_destroy(sim):
    _check(None, lib.gp_destroy(sim))


def _buffer(arr):
    """(pointer, dtype code, on_device) of a contiguous torch tensor or numpy array."""
    try:
        import torch
        if isinstance(arr, torch.Tensor):
            if not arr.is_contiguous():
                raise ValueError("tensor must be contiguous")
            code = {torch.float64: GP_FP64, torch.float32: GP_FP32}[arr.dtype]
            return ctypes.c_void_p(arr.data_ptr()), code, 1 if arr.is_cuda else 0
    except ImportError:
        pass
    if not (isinstance(arr, np.ndarray) and arr.flags["C_CONTIGUOUS"]):
        raise ValueError("need a C-contiguous numpy array or a contiguous torch tensor")
    code = {np.dtype(np.float64): GP_FP64, np.dtype(np.float32): GP_FP32}[arr.dtype]
    return ctypes.c_void_p(arr.ctypes.data), code, 0


def gp_set_field(sim, field, src):
    p, code, dev = _buffer(src)
    _check(sim, lib.gp_set_field(sim, int(field), p, code, dev))


def gp_get_field(sim, field, dst):
    p, code, dev = _buffer(dst)
    _check(sim, lib.gp_get_field(sim, int(field), p, code, dev))
    return dst


def gp_get_potential(sim, dst):
    p, code, dev = _buffer(dst)
    _check(sim, lib.gp_get_potential(sim, p, code, dev))
    return dst


def gp_potential_noalloc(cfg, rho, n, phi, stream=None):
    """Periodic potential of the device densities rho and n (FP64) into the
    device buffer phi (the config's precision), with no device allocation;
    enqueued on `stream` (a hipStream_t handle, None for the null stream)."""
    c = cfg if isinstance(cfg, gp_config) else make_config(cfg)
    (pr, cr, dr), (pn, cn, dn), (pp, cp, dp) = _buffer(rho), _buffer(n), _buffer(phi)
    if not (dr and dn and dp):
        raise ValueError("gp_potential_noalloc takes device buffers only")
    if cr != GP_FP64 or cn != GP_FP64 or cp != c.precision:
        raise ValueError("densities must be FP64 and phi of the config's precision")
    _check(None, lib.gp_potential_noalloc(ctypes.byref(c), pr, pn, pp, stream))
    return phi


def gp_step(sim, nsteps=1):
    _check(sim, lib.gp_step(sim, int(nsteps)))


def gp_sync(sim):
    _check(sim, lib.gp_sync(sim))


def gp_get_diag(sim, max_records=4096):
    buf = (gp_diag * max_records)()
    cnt = ctypes.c_int32()
    _check(sim, lib.gp_get_diag(sim, buf, max_records, ctypes.byref(cnt)))
    return _diag_dicts(buf, cnt.value)


def gp_set_time(sim, t, step=0):
    _check(sim, lib.gp_set_time(sim, float(t), int(step)))


def gp_get_time(sim):
    t, dt, st = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(sim, lib.gp_get_time(sim, ctypes.byref(t), ctypes.byref(dt), ctypes.byref(st)))
    return t.value, dt.value, st.value


def gp_debug_stage(sim, stage):
    _check(sim, lib.gp_debug_stage(sim, int(stage)))


def gp_time_kernels(sim, nsteps):
    ms = (ctypes.c_double * len(KERNEL_NAMES))()
    _check(sim, lib.gp_time_kernels(sim, int(nsteps), ms, len(KERNEL_NAMES)))
    return dict(zip(KERNEL_NAMES, list(ms)))


def gp_use_graph(sim, enable):
    _check(sim, lib.gp_use_graph(sim, 1 if enable else 0))


def gp_algorithmic_bytes_per_cell(sim, kernel=-1):
    return float(lib.gp_algorithmic_bytes_per_cell(sim, int(kernel)))


def gp_set_launch(sim, kernel, blocks):
    _check(sim, lib.gp_set_launch(sim, int(kernel), int(blocks)))


def gp_set_fft_form(sim, form):
    _check(sim, lib.gp_set_fft_form(sim, int(form)))


def gp_get_launch(sim, kernel):
    v = ctypes.c_int32()
    _check(sim, lib.gp_get_launch(sim, int(kernel), ctypes.byref(v)))
    return v.value


def gp_set_tiling(sim, kernel, shape, cap_planes):
    _check(sim, lib.gp_set_tiling(sim, int(kernel), int(shape), int(cap_planes)))


def gp_get_tiling(sim, kernel):
    s, c = ctypes.c_int32(), ctypes.c_int32()
    _check(sim, lib.gp_get_tiling(sim, int(kernel), ctypes.byref(s), ctypes.byref(c)))
    return s.value, c.value


def _diag_dicts(buf, n):
    out = []
    for r in buf[:n]:
        d = {k: getattr(r, k) for k, _ in gp_diag._fields_ if k not in ("mom", "pad")}
        d["mom_x"], d["mom_y"], d["mom_z"] = r.mom[0], r.mom[1], r.mom[2]
        out.append(d)
    return out


def gp_batch_create(cfgs, stream=None):
    arr = (gp_config * len(cfgs))(*[c if isinstance(c, gp_config) else make_config(c) for c in cfgs])
    h = ctypes.c_void_p()
    _check(None, lib.gp_batch_create(arr, len(cfgs), stream, ctypes.byref(h)), create=True)
    return h


def gp_batch_destroy(b):
    _check(None, lib.gp_batch_destroy(b))


def gp_batch_set_field(b, run, field, src):
    p, code, dev = _buffer(src)
    _check(b, lib.gp_batch_set_field(b, int(run), int(field), p, code, dev), True)


def gp_batch_get_field(b, run, field, dst):
    p, code, dev = _buffer(dst)
    _check(b, lib.gp_batch_get_field(b, int(run), int(field), p, code, dev), True)
    return dst


def gp_batch_get_potential(b, run, dst):
    p, code, dev = _buffer(dst)
    _check(b, lib.gp_batch_get_potential(b, int(run), p, code, dev), True)
    return dst


def gp_batch_step(b, nsteps=1):
    _check(b, lib.gp_batch_step(b, int(nsteps)), True)


def gp_batch_sync(b):
    _check(b, lib.gp_batch_sync(b), True)


def gp_batch_get_diag(b, run, max_records=4096):
    buf = (gp_diag * max_records)()
    cnt = ctypes.c_int32()
    _check(b, lib.gp_batch_get_diag(b, int(run), buf, max_records, ctypes.byref(cnt)), True)
    return _diag_dicts(buf, cnt.value)


def gp_batch_time_kernels(b, nsteps):
    ms = (ctypes.c_double * len(KERNEL_NAMES))()
    _check(b, lib.gp_batch_time_kernels(b, int(nsteps), ms, len(KERNEL_NAMES)), True)
    return dict(zip(KERNEL_NAMES, list(ms)))


def gp_batch_set_launch(b, kernel, blocks):
    _check(b, lib.gp_batch_set_launch(b, int(kernel), int(blocks)), True)


def gp_batch_set_fft_form(b, form):
    _check(b, lib.gp_batch_set_fft_form(b, int(form)), True)


def gp_batch_get_launch(b, kernel):
    v = ctypes.c_int32()
    _check(b, lib.gp_batch_get_launch(b, int(kernel), ctypes.byref(v)), True)
    return v.value


def gp_batch_set_tiling(b, kernel, shape, cap_planes):
    _check(b, lib.gp_batch_set_tiling(b, int(kernel), int(shape), int(cap_planes)), True)


def gp_batch_get_tiling(b, kernel):
    s, c = ctypes.c_int32(), ctypes.c_int32()
    _check(b, lib.gp_batch_get_tiling(b, int(kernel), ctypes.byref(s), ctypes.byref(c)), True)
    return s.value, c.value


def gp_batch_algorithmic_bytes_per_cell(b, kernel=-1):
    return float(lib.gp_batch_algorithmic_bytes_per_cell(b, int(kernel)))


def gp_batch_cells(b):
    return int(lib.gp_batch_cells(b))


class Sim:
    """One simulation on the current torch device and stream."""

    def __init__(self, cfg, stream=None):
        import torch
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        self.cfg = dict(cfg)
        self.shape = (int(cfg["n"][2]), int(cfg["n"][1]), int(cfg["n"][0]))
        self._h = gp_create(cfg, ctypes.c_void_p(stream) if stream else None)

    def close(self):
        if self._h is not None:
            gp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_field(self, name, src):
        import torch
        if isinstance(src, torch.Tensor) and src.is_cuda:
            torch.cuda.current_stream().synchronize()  # the producer may run on another stream
        gp_set_field(self._h, FIELD_NAMES.index(name) if isinstance(name, str) else name, src)

    def set_state(self, state):
        for k, v in state.items():
            self.set_field(k, v)

    def get_field(self, name, out=None, device="cuda", dtype=None):
        import torch
        fid = GP_PHI if name == "phi" else (FIELD_NAMES.index(name) if isinstance(name, str) else name)
        if out is None:
            out = torch.empty(self.shape, dtype=dtype or torch.float64, device=device)
        return gp_get_field(self._h, fid, out)

    def get_state(self, device="cuda", dtype=None):
        return {k: self.get_field(k, device=device, dtype=dtype) for k in FIELD_NAMES}

    def get_potential(self, out=None, device="cuda", dtype=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=dtype or torch.float64, device=device)
        return gp_get_potential(self._h, out)

    def step(self, n=1):
        gp_step(self._h, n)

    def sync(self):
        gp_sync(self._h)

    def stage(self, st):
        gp_debug_stage(self._h, st)

    def diag(self):
        return gp_get_diag(self._h)

    def time(self):
        return gp_get_time(self._h)

    def set_time(self, t, step=0):
        gp_set_time(self._h, t, step)

    def time_kernels(self, nsteps):
        return gp_time_kernels(self._h, nsteps)

    def use_graph(self, enable):
        gp_use_graph(self._h, enable)

    def bytes_per_cell(self, kernel=-1):
        return gp_algorithmic_bytes_per_cell(self._h, kernel)

    def set_launch(self, kernel, blocks):
        gp_set_launch(self._h, KERNEL_NAMES.index(kernel) if isinstance(kernel, str) else kernel, blocks)

    def set_fft_form(self, form):
        gp_set_fft_form(self._h, form)

    def get_launch(self, kernel):
        return gp_get_launch(self._h, KERNEL_NAMES.index(kernel) if isinstance(kernel, str) else kernel)

    def set_tiling(self, kernel, shape, cap_planes):
        gp_set_tiling(self._h, KERNEL_NAMES.index(kernel) if isinstance(kernel, str) else kernel, shape, cap_planes)

    def get_tiling(self, kernel):
        """(tile shape: 0 = 64 x 4, 1 = 32 x 8; z-chunk cap in planes)"""
        return gp_get_tiling(self._h, KERNEL_NAMES.index(kernel) if isinstance(kernel, str) else kernel)


class Batch:
    """An ensemble of independent runs advanced together (one precision)."""

    def __init__(self, cfgs, stream=None):
        import torch
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        self.cfgs = [dict(c) for c in cfgs]
        self.shapes = [(int(c["n"][2]), int(c["n"][1]), int(c["n"][0])) for c in cfgs]
        self._h = gp_batch_create(cfgs, ctypes.c_void_p(stream) if stream else None)

    def close(self):
        if self._h is not None:
            gp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.cfgs)

    def set_field(self, run, name, src):
        import torch
        if isinstance(src, torch.Tensor) and src.is_cuda:
            torch.cuda.current_stream().synchronize()
        gp_batch_set_field(self._h, run, FIELD_NAMES.index(name) if isinstance(name, str) else name, src)

    def set_state(self, run, state):
        for k, v in state.items():
            self.set_field(run, k, v)

    def get_field(self, run, name, out=None, device="cuda", dtype=None):
        import torch
        fid = GP_PHI if name == "phi" else (FIELD_NAMES.index(name) if isinstance(name, str) else name)
        if out is None:
            out = torch.empty(self.shapes[run], dtype=dtype or torch.float64, device=device)
        return gp_batch_get_field(self._h, run, fid, out)

    def get_state(self, run, device="cuda", dtype=None):
        return {k: self.get_field(run, k, device=device, dtype=dtype) for k in FIELD_NAMES}

    def get_potential(self, run, out=None, device="cuda", dtype=None):
        import torch
        if out is None:
            out = torch.empty(self.shapes[run], dtype=dtype or torch.float64, device=device)
        return gp_batch_get_potential(self._h, run, out)

    def step(self, n=1):
        gp_batch_step(self._h, n)

    def sync(self):
        gp_batch_sync(self._h)

    def diag(self, run):
        return gp_batch_get_diag(self._h, run)

    def time_kernels(self, nsteps):
        return gp_batch_time_kernels(self._h, nsteps)

    def set_launch(self, kernel, blocks):
        gp_batch_set_launch(self._h, KERNEL_NAMES.index(kernel) if isinstance(kernel, str) else kernel, blocks)

    def set_fft_form(self, form):
        gp_batch_set_fft_form(self._h, form)

    def get_launch(self, kernel):
        return gp_batch_get_launch(self._h, KERNEL_NAMES.index(kernel) if isinstance(kernel, str) else kernel)

    def set_tiling(self, kernel, shape, cap_planes):
        gp_batch_set_tiling(self._h, KERNEL_NAMES.index(kernel) if isinstance(kernel, str) else kernel, shape,
                            cap_planes)

    def get_tiling(self, kernel):
        return gp_batch_get_tiling(self._h, KERNEL_NAMES.index(kernel) if isinstance(kernel, str) else kernel)

    def bytes_per_cell(self, kernel=-1):
        return gp_batch_algorithmic_bytes_per_cell(self._h, kernel)

    def cells(self):
        return gp_batch_cells(self._h)
