"""ctypes binding of libacch.so (include/acch.h): argument marshalling only.

Every stage of the time step runs in the HIP library; PyTorch provides the device
workspace and the stream.  If the library has not been built the binding raises —
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libacch.so")

ACCH_OK, ACCH_EINVAL, ACCH_EDOMAIN, ACCH_EDIVERGED, ACCH_EDEVICE, ACCH_EUNSUPPORTED = range(6)
EXPORT_JACOBIAN, EXPORT_FACTORS, EXPORT_BOXES, EXPORT_BAND = 0, 1, 2, 3

EXPORTED = [
    "acch_params_default", "acch_workspace_bytes", "acch_create", "acch_step", "acch_energy",
    "acch_destroy", "acch_get_fields", "acch_set_fields", "acch_get_time", "acch_residual",
    "acch_jacobian", "acch_apply_jacobian", "acch_factor", "acch_precondition", "acch_gmres",
    "acch_solve_step", "acch_export", "acch_info", "acch_strerror", "acch_last_error",
    "acch_timing", "acch_kernel_stats", "acch_counters", "acch_set_option",
    "acch_apply_jacobian_transpose", "acch_precondition_transpose", "acch_energy_gradient", "acch_adjoint_step",
    "acch_batch_workspace_bytes", "acch_batch_create", "acch_batch_step", "acch_batch_energy",
    "acch_batch_get_fields", "acch_batch_set_option", "acch_batch_counters", "acch_batch_destroy",
    "acch_batch_precondition", "acch_batch_info", "acch_residual_noalloc",
]
KERNEL_KINDS = ["residual", "jacobian", "factor", "ras", "spmv_dots", "orth", "gmres_start", "gmres_update",
                "energy", "spmv", "other"]


class Params(ctypes.Structure):
    """Mirror of acch_params."""
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("L", ctypes.c_double * 3), ("bc", ctypes.c_int),
        ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("theta", ctypes.c_double),
        ("gamma", ctypes.c_double), ("rho", ctypes.c_double), ("S", ctypes.c_int), ("adaptive", ctypes.c_int),
        ("dt_fixed", ctypes.c_double), ("dt_min", ctypes.c_double), ("dt_max", ctypes.c_double),
        ("eta0", ctypes.c_double), ("newton_rtol", ctypes.c_double), ("newton_atol", ctypes.c_double),
        ("newton_max_it", ctypes.c_int), ("gmres_rtol", ctypes.c_double), ("gmres_atol", ctypes.c_double),
        ("gmres_restart", ctypes.c_int), ("gmres_max_restarts", ctypes.c_int), ("ras_type", ctypes.c_int),
        ("sub", ctypes.c_int * 3), ("overlap", ctypes.c_int), ("ilu_reuse", ctypes.c_int),
        ("precision", ctypes.c_int), ("mobility_mode", ctypes.c_int), ("xd_norm", ctypes.c_int),
        ("mass_projection", ctypes.c_int), ("log_energy", ctypes.c_int), ("ilu_shift", ctypes.c_double),
        ("subsolver", ctypes.c_int), ("fill_level", ctypes.c_int),
        ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t), ("stream", ctypes.c_void_p),
    ]


class StepInfo(ctypes.Structure):
    """Mirror of acch_step_info."""
    _fields_ = [
        ("t", ctypes.c_double), ("dt", ctypes.c_double), ("eta", ctypes.c_double), ("energy", ctypes.c_double),
        ("mass", ctypes.c_double), ("fnorm", ctypes.c_double), ("newton_its", ctypes.c_int),
        ("gmres_its", ctypes.c_int), ("retries", ctypes.c_int), ("status", ctypes.c_int),
    ]

    def as_dict(self) -> Dict[str, float]:
        return {name: getattr(self, name) for name, _ in self._fields_}


class AcchError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"acch error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libacch.so (built by paper_2007_04560_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2007_04560_amd.build` "
                           "(the solver has no non-HIP fallback)")
    lib = ctypes.CDLL(p)
    vp, dp, ip, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_size_t
    ctx = ctypes.c_void_p
    sig = {
        "acch_params_default": (None, [ctypes.POINTER(Params)]),
        "acch_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(sz)]),
        "acch_create": (ctypes.c_int, [ctypes.POINTER(Params), vp, vp, ctypes.POINTER(ctx)]),
        "acch_step": (ctypes.c_int, [ctx, ctypes.c_int, ctypes.POINTER(StepInfo), ip]),
        "acch_energy": (ctypes.c_int, [ctx, dp, dp]),
        "acch_destroy": (ctypes.c_int, [ctx]),
        "acch_get_fields": (ctypes.c_int, [ctx, vp, vp]),
        "acch_set_fields": (ctypes.c_int, [ctx, vp, vp]),
        "acch_get_time": (ctypes.c_int, [ctx, dp, dp, dp]),
        "acch_residual": (ctypes.c_int, [ctx, vp, vp, ctypes.c_double, vp, dp, ip]),
        "acch_residual_noalloc": (ctypes.c_int, [ctypes.POINTER(Params), vp, vp, ctypes.c_double, vp, dp, ip]),
        "acch_jacobian": (ctypes.c_int, [ctx, vp, vp, ctypes.c_double]),
        "acch_apply_jacobian": (ctypes.c_int, [ctx, vp, vp]),
        "acch_factor": (ctypes.c_int, [ctx]),
        "acch_precondition": (ctypes.c_int, [ctx, vp, vp]),
        "acch_gmres": (ctypes.c_int, [ctx, vp, vp, ip, dp]),
        "acch_solve_step": (ctypes.c_int, [ctx, ctypes.c_double, ctypes.POINTER(StepInfo)]),
        "acch_export": (ctypes.c_int, [ctx, ctypes.c_int, vp, ctypes.POINTER(sz)]),
        "acch_info": (ctypes.c_int, [ctx, ctypes.POINTER(ctypes.c_long), ip, ip, ip]),
        "acch_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "acch_last_error": (ctypes.c_char_p, []),
        "acch_timing": (ctypes.c_int, [ctx, ctypes.c_int]),
        "acch_kernel_stats": (ctypes.c_int, [ctx, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_long)]),
        "acch_counters": (ctypes.c_int, [ctx, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]),
        "acch_set_option": (ctypes.c_int, [ctx, ctypes.c_int, ctypes.c_long]),
        "acch_apply_jacobian_transpose": (ctypes.c_int, [ctx, vp, vp]),
        "acch_precondition_transpose": (ctypes.c_int, [ctx, vp, vp]),
        "acch_energy_gradient": (ctypes.c_int, [ctx, vp, vp, dp]),
        "acch_adjoint_step": (ctypes.c_int, [ctx, vp, vp, ctypes.c_double, vp, vp, dp, ip, dp]),
        "acch_batch_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(sz)]),
        "acch_batch_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int, vp, vp, ctypes.POINTER(ctx)]),
        "acch_batch_step": (ctypes.c_int, [ctx, ctypes.c_int, ip, ip]),
        "acch_batch_energy": (ctypes.c_int, [ctx, dp, dp]),
        "acch_batch_get_fields": (ctypes.c_int, [ctx, ctypes.c_int, vp, vp]),
        "acch_batch_set_option": (ctypes.c_int, [ctx, ctypes.c_int, ctypes.c_long]),
        "acch_batch_counters": (ctypes.c_int, [ctx, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long),
                                               ctypes.POINTER(ctypes.c_long)]),
        "acch_batch_destroy": (ctypes.c_int, [ctx]),
        "acch_batch_precondition": (ctypes.c_int, [ctx, vp, vp]),
        "acch_batch_info": (ctypes.c_int, [ctx, ctypes.POINTER(ctypes.c_long), ip, ip, ip,
                                           ctypes.POINTER(ctypes.c_long)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(lib, rc: int):
    if rc != ACCH_OK:
        raise AcchError(rc, f"{lib.acch_strerror(rc).decode()}: {lib.acch_last_error().decode()}")


_OPTIONS = {"ras_prefetch": 0, "ras3d_window": 1}


def set_option(name: str, value: int):
    """Process-wide tuning option of the library (acch_set_option): "ras_prefetch"
    (2D triangular-solve prefetch depth) or "ras3d_window" (1: keep the recent levels
    of a 3D box in LDS when it fits, 0: whole box in device memory)."""
    lib = load_library()
    _check(lib, lib.acch_set_option(None, _OPTIONS[name], int(value)))


_BC = {"periodic": 0, "neumann": 1}
_SCHWARZ = {"left": 0, "right": 1, "classical": 2}
_PREC = {"fp64": 0, "mixed": 1}
_MOB = {"midpoint": 0, "average": 1, "explicit": 2}
_SUBSOLVER = {"ilu0": 0, "iluk": 1, "lu": 2, "iluk_box": 3}


def make_params(shape: Sequence[int], *, bc="periodic", L=(1.0, 1.0), alpha=1.2, beta=1.2, theta=0.1,
                gamma=1e-3, rho=1.0, S=10, adaptive=False, dt_fixed=1e-3, dt_min=1e-4, dt_max=1e-1, eta0=1e4,
                newton_rtol=1e-8, newton_atol=1e-13, newton_max_it=50, gmres_rtol=1e-8, gmres_atol=1e-14,
                gmres_restart=30, gmres_max_restarts=10, sub=(2, 2), overlap=1, ilu_reuse=True,
                precision="fp64", mobility="midpoint", xd_norm="plain", mass_projection=True,
                log_energy=True, ilu_shift=0.0, schwarz="left", subsolver="ilu0", fill_level=0) -> Params:
    """acch_params for a 2D field of shape (ny, nx) or a 3D field of shape (nz, ny, nx);
    L and sub are given in x, y[, z] order."""
    p = Params()
    if len(shape) == 3:
        nz, ny, nx = int(shape[0]), int(shape[1]), int(shape[2])
        p.dim = 3
    else:
        ny, nx = int(shape[0]), int(shape[1])
        nz = 1
        p.dim = 2
    p.n[0], p.n[1], p.n[2] = nx, ny, nz
    p.L[0], p.L[1] = float(L[0]), float(L[1])
    p.L[2] = float(L[2]) if len(L) > 2 else 1.0
    p.bc = _BC[bc]
    p.alpha, p.beta, p.theta, p.gamma, p.rho = alpha, beta, theta, gamma, rho
    p.S = S
    p.adaptive = int(bool(adaptive))
    p.dt_fixed, p.dt_min, p.dt_max, p.eta0 = dt_fixed, dt_min, dt_max, eta0
    p.newton_rtol, p.newton_atol, p.newton_max_it = newton_rtol, newton_atol, newton_max_it
    p.gmres_rtol, p.gmres_atol = gmres_rtol, gmres_atol
    p.gmres_restart, p.gmres_max_restarts = gmres_restart, gmres_max_restarts
    p.ras_type = _SCHWARZ[schwarz]
    p.sub[0], p.sub[1], p.sub[2] = int(sub[0]), int(sub[1]), int(sub[2]) if len(sub) > 2 else 1
    p.overlap = overlap
    p.ilu_reuse = 1 if ilu_reuse else -1
    p.precision = _PREC[precision]
    p.mobility_mode = _MOB[mobility]
    p.xd_norm = 0 if xd_norm == "plain" else 1
    p.mass_projection = 1 if mass_projection else -1
    p.log_energy = 1 if log_energy else -1
    p.ilu_shift = float(ilu_shift)
    p.subsolver = _SUBSOLVER[subsolver]
    p.fill_level = int(fill_level)
    return p


def _ptr(t) -> int:
    return t.data_ptr()


class Solver:
    """One 2D problem on the current GPU: owns the torch workspace and the acch context."""

    def __init__(self, u0: np.ndarray, v0: np.ndarray, device=None, **kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("acch needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        if u0.shape != v0.shape or u0.ndim not in (2, 3):
            raise ValueError("u0 and v0 must be arrays of one shape, (ny, nx) or (nz, ny, nx)")
        self.shape = u0.shape
        self.ncell = int(u0.size)
        self.params = make_params(self.shape, **kw)
        nbytes = ctypes.c_size_t(0)
        _check(self.lib, self.lib.acch_workspace_bytes(ctypes.byref(self.params), ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self._ws_raw = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        base = self._ws_raw.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.params.workspace = aligned
        self.params.workspace_bytes = self.workspace_bytes
        self.params.stream = self.stream.cuda_stream
        self.ctx = ctypes.c_void_p()
        _check(self.lib, self.lib.acch_create(ctypes.byref(self.params), u0.ctypes.data, v0.ctypes.data,
                                              ctypes.byref(self.ctx)))

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self.lib.acch_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- time stepping ----------------------------------------------------------
    def step(self, nsteps: int = 1) -> List[Dict[str, float]]:
        info = (StepInfo * max(1, nsteps))()
        acc = ctypes.c_int(0)
        rc = self.lib.acch_step(self.ctx, nsteps, info, ctypes.byref(acc))
        self.last_accepted = [info[k].as_dict() for k in range(acc.value)]
        _check(self.lib, rc)
        return self.last_accepted

    def solve_step(self, dt: float) -> Dict[str, float]:
        info = StepInfo()
        _check(self.lib, self.lib.acch_solve_step(self.ctx, dt, ctypes.byref(info)))
        return info.as_dict()

    def energy(self) -> Tuple[float, float]:
        e, m = ctypes.c_double(), ctypes.c_double()
        _check(self.lib, self.lib.acch_energy(self.ctx, ctypes.byref(e), ctypes.byref(m)))
        return e.value, m.value

    def fields(self) -> Tuple[np.ndarray, np.ndarray]:
        u = np.empty(self.shape)
        v = np.empty(self.shape)
        _check(self.lib, self.lib.acch_get_fields(self.ctx, u.ctypes.data, v.ctypes.data))
        return u, v

    def set_fields(self, u: np.ndarray, v: np.ndarray):
        u = np.ascontiguousarray(u, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        _check(self.lib, self.lib.acch_set_fields(self.ctx, u.ctypes.data, v.ctypes.data))

    def time(self) -> Tuple[float, float, float]:
        t, dtp, eta = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self.lib, self.lib.acch_get_time(self.ctx, ctypes.byref(t), ctypes.byref(dtp), ctypes.byref(eta)))
        return t.value, dtp.value, eta.value

    def timing(self, enable=True):
        """True / 1: time every launch; 2: sample the Schwarz launches only (acch_timing)."""
        _check(self.lib, self.lib.acch_timing(self.ctx, 2 if enable == 2 else int(bool(enable))))

    def kernel_stats(self) -> Dict[str, Tuple[float, int]]:
        out = {}
        for k, name in enumerate(KERNEL_KINDS):
            ms, cnt = ctypes.c_double(), ctypes.c_long()
            _check(self.lib, self.lib.acch_kernel_stats(self.ctx, k, ctypes.byref(ms), ctypes.byref(cnt)))
            out[name] = (ms.value, cnt.value)
        return out

    def counters(self) -> Tuple[int, int]:
        a, b = ctypes.c_long(), ctypes.c_long()
        _check(self.lib, self.lib.acch_counters(self.ctx, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def info(self):
        n, ns, bw, bh = ctypes.c_long(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self.lib, self.lib.acch_info(self.ctx, ctypes.byref(n), ctypes.byref(ns), ctypes.byref(bw),
                                            ctypes.byref(bh)))
        return {"ncell": n.value, "nsub": ns.value, "box_w": bw.value, "box_h": bh.value}

    # -- operator-level entry points (device tensors of 2*ncell doubles) --------
    def vector(self, X=None):
        t = self.torch
        if X is None:
            return t.empty(2 * self.ncell, dtype=t.float64, device=self.device)
        return t.as_tensor(np.ascontiguousarray(X, dtype=np.float64)).to(self.device)

    def residual(self, X, Xn, dt: float):
        F = self.vector()
        f2 = ctypes.c_double()
        bad = ctypes.c_int()
        _check(self.lib, self.lib.acch_residual(self.ctx, _ptr(X), _ptr(Xn), dt, _ptr(F), ctypes.byref(f2),
                                                ctypes.byref(bad)))
        return F, f2.value, bad.value

    def jacobian(self, X, Xn, dt: float):
        _check(self.lib, self.lib.acch_jacobian(self.ctx, _ptr(X), _ptr(Xn), dt))

    def apply_jacobian(self, x):
        y = self.vector()
        _check(self.lib, self.lib.acch_apply_jacobian(self.ctx, _ptr(x), _ptr(y)))
        return y

    def factor(self):
        _check(self.lib, self.lib.acch_factor(self.ctx))

    def precondition(self, r):
        z = self.vector()
        _check(self.lib, self.lib.acch_precondition(self.ctx, _ptr(r), _ptr(z)))
        return z

    def gmres(self, F):
        S = self.vector()
        its = ctypes.c_int()
        res = ctypes.c_double()
        _check(self.lib, self.lib.acch_gmres(self.ctx, _ptr(F), _ptr(S), ctypes.byref(its), ctypes.byref(res)))
        return S, its.value, res.value

    # -- discrete adjoint (device tensors of 2*ncell doubles) -------------------
    def apply_jacobian_transpose(self, x):
        y = self.vector()
        _check(self.lib, self.lib.acch_apply_jacobian_transpose(self.ctx, _ptr(x), _ptr(y)))
        return y

    def precondition_transpose(self, r):
        z = self.vector()
        _check(self.lib, self.lib.acch_precondition_transpose(self.ctx, _ptr(r), _ptr(z)))
        return z

    def energy_gradient(self, X=None):
        """(dE~/dX as a device tensor, dE~/d(alpha, beta, theta, gamma) as a float64 array)."""
        g = self.vector()
        dp = (ctypes.c_double * 4)()
        _check(self.lib, self.lib.acch_energy_gradient(self.ctx, None if X is None else _ptr(X), _ptr(g), dp))
        return g, np.array(dp[:], dtype=np.float64)

    def adjoint_step(self, X1, X0, dt: float, g, dparams=None, out=None):
        """One step back through F(X1; X0, dt) = 0: returns (dL/dX0, dparams updated by
        -lambda . dF/dp, GMRES iterations, residual estimate)."""
        out = self.vector() if out is None else out
        acc = np.zeros(4) if dparams is None else np.array(dparams, dtype=np.float64)
        dp = (ctypes.c_double * 4)(*acc.tolist())
        its = ctypes.c_int()
        res = ctypes.c_double()
        _check(self.lib, self.lib.acch_adjoint_step(self.ctx, _ptr(X1), _ptr(X0), dt, _ptr(g), _ptr(out), dp,
                                                    ctypes.byref(its), ctypes.byref(res)))
        return out, np.array(dp[:], dtype=np.float64), its.value, res.value

    def _export(self, which, dtype):
        t = self.torch
        nb = ctypes.c_size_t(0)
        _check(self.lib, self.lib.acch_export(self.ctx, which, None, ctypes.byref(nb)))
        out = t.empty(int(nb.value) // np.dtype(dtype).itemsize, dtype=getattr(t, np.dtype(dtype).name),
                      device=self.device)
        _check(self.lib, self.lib.acch_export(self.ctx, which, _ptr(out), ctypes.byref(nb)))
        return out

    def export_jacobian(self):
        nslot = 40 if len(self.shape) == 3 else 24
        return self._export(EXPORT_JACOBIAN, np.float64).reshape((nslot,) + tuple(self.shape))

    def export_factors(self):
        i = self.info()
        if self.params.subsolver == _SUBSOLVER["iluk_box"] and self.params.fill_level == 0:
            # box-pattern ILU(0): [sub][cell j*bw + i][L record (52), U record (52)]
            return self._export(EXPORT_FACTORS, np.float64).reshape(i["nsub"], i["box_w"] * i["box_h"], 104)
        if len(self.shape) == 3:
            return self._export(EXPORT_FACTORS, np.float64).reshape(i["nsub"], 40, -1)
        return self._export(EXPORT_FACTORS, np.float64).reshape(i["nsub"], 24, i["box_h"], i["box_w"])

    def export_boxes(self):
        return self._export(EXPORT_BOXES, np.int32).reshape(-1, 4)

    def export_band(self):
        """ILU(k) / exact-LU factors [sub][R][d] (include/acch.h, ACCH_EXPORT_BAND)."""
        i = self.info()
        n = 2 * i["box_w"] * i["box_h"]
        return self._export(EXPORT_BAND, np.float64).reshape(i["nsub"], n, -1)   # 2 kl + 1 diagonals


class BatchSolver:
    """Many independent instances advanced together by acch_batch_* (one launch per
    stage for all instances).  ``fields`` is a list of (u0, v0) host arrays, ``params``
    a list of per-instance keyword dicts for make_params (bc, L, alpha, ..., sub);
    ``common`` holds the settings shared by the batch (dt_fixed, tolerances,
    precision, overlap, ilu_shift, and the subdomain solver: ILU(0) on the stencil
    pattern, or subsolver="iluk_box" with fill_level=0 for ILU(0) on the box pattern).
    The batch runs on its own created stream so that its GMRES cycles can be recorded
    into HIP graphs."""

    def __init__(self, fields, params=None, device=None, graph: bool = True, **common):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("acch needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.torch = torch
        self.count = len(fields)
        params = params or [{} for _ in fields]
        if len(params) != self.count:
            raise ValueError("one parameter dict per instance")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._u = [np.ascontiguousarray(u, dtype=np.float64) for u, _ in fields]
        self._v = [np.ascontiguousarray(v, dtype=np.float64) for _, v in fields]
        self.shapes = [u.shape for u in self._u]
        arr = (Params * self.count)()
        for i in range(self.count):
            kw = dict(common)
            kw.update(params[i])
            arr[i] = make_params(self.shapes[i], **kw)
        self.params = arr
        nbytes = ctypes.c_size_t(0)
        _check(self.lib, self.lib.acch_batch_workspace_bytes(arr, self.count, ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self._ws_raw = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.Stream(device=self.device)
        base = self._ws_raw.data_ptr()
        arr[0].workspace = (base + 255) // 256 * 256
        arr[0].workspace_bytes = self.workspace_bytes
        arr[0].stream = self.stream.cuda_stream
        pu = (ctypes.c_void_p * self.count)(*[u.ctypes.data for u in self._u])
        pv = (ctypes.c_void_p * self.count)(*[v.ctypes.data for v in self._v])
        self.ctx = ctypes.c_void_p()
        # the workspace tensor was made on the current stream: finish before the batch stream uses it
        torch.cuda.current_stream(self.device).synchronize()
        _check(self.lib, self.lib.acch_batch_create(arr, self.count, pu, pv, ctypes.byref(self.ctx)))
        self.set_graph(graph)   # records the cycle graphs now when on

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self.lib.acch_batch_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_graph(self, enable: bool):
        _check(self.lib, self.lib.acch_batch_set_option(self.ctx, 0, int(bool(enable))))

    def step(self, nsteps: int = 1):
        """Returns per-instance Newton and GMRES iteration counts of these steps."""
        nit = (ctypes.c_int * self.count)()
        git = (ctypes.c_int * self.count)()
        _check(self.lib, self.lib.acch_batch_step(self.ctx, nsteps, nit, git))
        return np.array(nit[:]), np.array(git[:])

    def energy(self):
        e = (ctypes.c_double * self.count)()
        m = (ctypes.c_double * self.count)()
        _check(self.lib, self.lib.acch_batch_energy(self.ctx, e, m))
        return np.array(e[:]), np.array(m[:])

    def fields(self, i: int):
        u = np.empty(self.shapes[i])
        v = np.empty(self.shapes[i])
        _check(self.lib, self.lib.acch_batch_get_fields(self.ctx, i, u.ctypes.data, v.ctypes.data))
        return u, v

    def info(self):
        n, ns, bw, bh = ctypes.c_long(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        xo = (ctypes.c_long * self.count)()
        _check(self.lib, self.lib.acch_batch_info(self.ctx, ctypes.byref(n), ctypes.byref(ns), ctypes.byref(bw),
                                                  ctypes.byref(bh), xo))
        return {"ncell": n.value, "nsub": ns.value, "box_w": bw.value, "box_h": bh.value, "xoff": list(xo[:])}

    def vector(self):
        return self.torch.empty(2 * self.info()["ncell"], dtype=self.torch.float64, device=self.device)

    def precondition(self, r, z=None):
        """z = M^{-1} r for all instances (batched device vectors), asynchronous on
        the batch stream."""
        z = self.vector() if z is None else z
        _check(self.lib, self.lib.acch_batch_precondition(self.ctx, _ptr(r), _ptr(z)))
        return z

    def counters(self):
        a, g, s = ctypes.c_long(), ctypes.c_long(), ctypes.c_long()
        _check(self.lib, self.lib.acch_batch_counters(self.ctx, ctypes.byref(a), ctypes.byref(g), ctypes.byref(s)))
        return {"launches": a.value, "graph_launches": g.value, "syncs": s.value}
