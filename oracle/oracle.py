"""ctypes binding of the FP64 CPU oracle (``gpupegas_oracle.c``).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline use it.  Arrays are numpy float64, shape (nz, ny, nx) in C order, so
x is the fastest index, matching the oracle's cell index i + nx (j + ny k).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpupegas_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FIELD_NAMES = [
    "rho", "mx", "my", "mz", "E", "e",
    "n", "qx", "qy", "qz",
    "Pxx", "Pxy", "Pxz", "Pyy", "Pyz", "Pzz",
    "Wxx", "Wxy", "Wxz", "Wyy", "Wyz", "Wzz",
]
PHI = 22
DIAG_FIELDS = [
    "step", "t", "dt", "mass_gas", "mass_bme", "mom_x", "mom_y", "mom_z",
    "e_gas", "e_bme", "e_pot", "kappa_gas", "kappa_bme", "outflow_gas",
    "outflow_bme", "n_sync_gas", "n_sync_bme", "err",
]

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
          "-shared", "-std=c11", "-D_DEFAULT_SOURCE", "-Wall"]


def lib_path():
    return _LIB


def build(force=True):
    """Compile the oracle with gcc (plain C, no contraction, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class OracleConfig(ctypes.Structure):
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
        ("poisson", ctypes.c_int32),
        ("cool_lambda", ctypes.c_double),
        ("cool_alpha", ctypes.c_double),
        ("cool_theta_min", ctypes.c_double),
        ("gext", ctypes.c_double * 3),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_create.restype = ctypes.c_void_p
    L.orc_create.argtypes = [ctypes.POINTER(OracleConfig)]
    L.orc_destroy.argtypes = [ctypes.c_void_p]
    L.orc_set_field.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    L.orc_get_field.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    L.orc_set_time.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int64]
    L.orc_get_dt.argtypes = [ctypes.c_void_p]
    L.orc_get_dt.restype = ctypes.c_double
    L.orc_stage.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_get_diag.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.orc_riemann_gas.argtypes = [ctypes.c_double] * 7 + [dp, dp]
    L.orc_riemann_bme.argtypes = [ctypes.c_double, dp, dp, ctypes.c_double, dp, dp,
                                  ctypes.c_int, dp, dp]
    L.orc_dft3.argtypes = [ctypes.c_int] * 3 + [dp, dp, ctypes.c_int]
    L.orc_poisson.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double, dp, dp]
    L.orc_poisson_isolated.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double, dp, dp]
    L.orc_get_phi_ext.argtypes = [ctypes.c_void_p, dp]
    L.orc_diag_count.argtypes = [ctypes.c_void_p]
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_get_threads.restype = ctypes.c_int
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n):
    _load().orc_set_threads(int(n))


def get_threads():
    return int(_load().orc_get_threads())


def riemann_gas(rl, vl, pl, rr, vr, pr, gamma):
    L = _load()
    V, P = ctypes.c_double(), ctypes.c_double()
    L.orc_riemann_gas(rl, vl, pl, rr, vr, pr, gamma, ctypes.byref(V), ctypes.byref(P))
    return V.value, P.value


def riemann_bme(nl, ul, pil, nr, ur, pir, d):
    """Face state for normal axis d; Pi given as 6 slots xx,xy,xz,yy,yz,zz.
    Returns (u*[3], Pi*_{d,:}[3]) in lab components."""
    L = _load()
    ul, pil, ur, pir = (np.ascontiguousarray(x, dtype=np.float64) for x in (ul, pil, ur, pir))
    us, ps = np.zeros(3), np.zeros(3)
    L.orc_riemann_bme(nl, _dp(ul), _dp(pil), nr, _dp(ur), _dp(pir), int(d), _dp(us), _dp(ps))
    return us, ps


def dft3(x, sign=-1):
    """Unnormalised 3D DFT of a complex array shaped (nz, ny, nx)."""
    L = _load()
    re = np.ascontiguousarray(np.real(x), dtype=np.float64).copy()
    im = np.ascontiguousarray(np.imag(x), dtype=np.float64).copy()
    nz, ny, nx = re.shape
    if L.orc_dft3(nx, ny, nz, _dp(re), _dp(im), int(sign)) != 0:
        raise ValueError("length not of the form 2^a 3^b")
    return re + 1j * im


def poisson(s, h, G=1.0):
    L = _load()
    s = np.ascontiguousarray(s, dtype=np.float64)
    nz, ny, nx = s.shape
    phi = np.zeros_like(s)
    if L.orc_poisson(nx, ny, nz, float(h), float(G), _dp(s), _dp(phi)) != 0:
        raise ValueError("length not of the form 2^a 3^b")
    return phi


def poisson_isolated(s, h, G=1.0):
    """Isolated potential of s (nz, ny, nx) on the grid and its one-cell
    ring: shape (nz + 2, ny + 2, nx + 2), cell i at index i + 1."""
    L = _load()
    s = np.ascontiguousarray(s, dtype=np.float64)
    nz, ny, nx = s.shape
    phi = np.zeros((nz + 2, ny + 2, nx + 2))
    if L.orc_poisson_isolated(nx, ny, nz, float(h), float(G), _dp(s), _dp(phi)) != 0:
        raise ValueError("length not of the form 2^a 3^b")
    return phi


class Oracle:
    """One oracle simulation.  ``cfg`` is a dict with keys n, lo, hi, gamma, G,
    cfl, eta, fixed_dt, t_end, bc (0 outflow, 1 periodic per axis), poisson
    ("periodic" / "isolated") and the cooling law cool_lambda, cool_alpha,
    cool_theta_min (absent: no cooling), and gext, a uniform external
    gravitational acceleration (absent: none)."""

    def __init__(self, cfg):
        L = _load()
        c = OracleConfig()
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
        c.poisson = {"periodic": 0, "isolated": 1}[cfg.get("poisson", "periodic")]
        c.cool_lambda = float(cfg.get("cool_lambda", 0.0))
        c.cool_alpha = float(cfg.get("cool_alpha", 0.0))
        c.cool_theta_min = float(cfg.get("cool_theta_min", 0.0))
        for d in range(3):
            c.gext[d] = float(cfg.get("gext", (0.0, 0.0, 0.0))[d])
        self._cfg = c
        self._h = L.orc_create(ctypes.byref(c))
        if not self._h:
            raise ValueError("invalid oracle configuration")
        self.shape = (c.n[2], c.n[1], c.n[0])
        self.h = (c.hi[0] - c.lo[0]) / c.n[0]
        self._L = L

    def close(self):
        if self._h:
            self._L.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_field(self, fid, arr):
        fid = FIELD_NAMES.index(fid) if isinstance(fid, str) else int(fid)
        a = np.ascontiguousarray(arr, dtype=np.float64)
        assert a.shape == self.shape, (a.shape, self.shape)
        if self._L.orc_set_field(self._h, fid, _dp(a)) != 0:
            raise ValueError("bad field id")

    def set_state(self, state):
        for k, v in state.items():
            self.set_field(k, v)

    def get_field(self, fid):
        fid = (PHI if fid == "phi" else FIELD_NAMES.index(fid)) if isinstance(fid, str) else int(fid)
        out = np.empty(self.shape, dtype=np.float64)
        if self._L.orc_get_field(self._h, fid, _dp(out)) != 0:
            raise ValueError("bad field id")
        return out

    def get_state(self):
        return {k: self.get_field(k) for k in FIELD_NAMES}

    def get_phi_ext(self):
        """Isolated potential on the grid and its one-cell ring."""
        out = np.empty(tuple(v + 2 for v in self.shape), dtype=np.float64)
        if self._L.orc_get_phi_ext(self._h, _dp(out)) != 0:
            raise ValueError("not an isolated-boundary run")
        return out

    def set_time(self, t, step=0):
        self._L.orc_set_time(self._h, float(t), int(step))

    def dt(self):
        return float(self._L.orc_get_dt(self._h))

    def stage(self, st):
        if self._L.orc_stage(self._h, int(st)) != 0:
            raise RuntimeError("stage out of order")

    def step(self, n=1):
        r = self._L.orc_step(self._h, int(n))
        if r < 0:
            raise RuntimeError("oracle step called mid-step")
        return r

    def diag(self):
        max_records = int(self._L.orc_diag_count(self._h))
        out = np.zeros((max(max_records, 1), len(DIAG_FIELDS)))
        cnt = ctypes.c_int()
        self._L.orc_get_diag(self._h, _dp(out), max_records, ctypes.byref(cnt))
        return [dict(zip(DIAG_FIELDS, row)) for row in out[: cnt.value]]
