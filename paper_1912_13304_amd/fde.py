"""ctypes binding of libfde (include/fde.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Vectors are torch float64 CUDA (HIP) tensors; their device
pointers and the current torch stream are handed to the C entry points.
The library must have been built (``paper_1912_13304_amd/build.py``); there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfde.so")

FDE_OK, FDE_ENOTCONV, FDE_EINVAL, FDE_ENOMEM, FDE_EHIP, FDE_ENONFINITE, FDE_EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "FDE_OK", 1: "FDE_ENOTCONV", -1: "FDE_EINVAL", -2: "FDE_ENOMEM", -3: "FDE_EHIP",
                -4: "FDE_ENONFINITE", -5: "FDE_EUNSUPPORTED"}
W_SHIFTED, W_WEIGHTED = 0, 1
T_EULER, T_CN = 0, 1
P_NONE, P_TAU, P_TAU_HAT, P_TILDE, P_TRI = 0, 1, 2, 3, 4
D_LEFT, D_RIGHT = 0, 1
S_GMRES, S_PCG = 0, 1
FP64, MIXED = 0, 1

PROBE_OFF, PROBE_MAXPY64, PROBE_MDOT64, PROBE_LINE64, PROBE_LINE32, PROBE_MAXPY32, PROBE_MDOT32, PROBE_CGS64, PROBE_CGS32 = range(9)
PROBE_LINE64_VARIANT, PROBE_LINE32_VARIANT = 64, 96
# line program flags (fde_lines.hpp): DST1 = 1, FDST2 = 2, STOREZ = 4, TOEP = 8, EXTBASE = 16
LINE_PROGRAMS = {1: "dst", 3: "dst_f_dst", 8: "toeplitz", 11: "dst_f_dst_toeplitz", 12: "storez_toeplitz",
                 13: "dst_storez_toeplitz", 15: "dst_f_dst_storez_toeplitz", 24: "toeplitz_base"}

EXPORTED = ["fde_default_params", "fde_assemble", "fde_matvec", "fde_tau_apply", "fde_matvec_f32",
            "fde_tau_apply_f32", "fde_solve", "fde_rhs",
            "fde_plan_bytes", "fde_destroy", "fde_release_cache", "fde_last_error", "fde_probe", "fde_probe_read",
            "fde_batch_layout", "fde_batch_bytes", "fde_batch_assemble", "fde_batch_solve", "fde_batch_run",
            "fde_batch_tune", "fde_batch_get_cfg", "fde_batch_set_cfg", "fde_batch_destroy",
            "fde_batch_matvec", "fde_batch_tau_apply", "fde_pcg1d_solve_noalloc"]
BATCH_VARIANTS = 4


class FdeParams(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int * 2),
        ("alpha", ctypes.c_double * 2),
        ("lo", ctypes.c_double * 2),
        ("hi", ctypes.c_double * 2),
        ("dt", ctypes.c_double),
        ("weights", ctypes.c_int),
        ("time", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("dside", ctypes.c_int),
        ("shift", ctypes.c_double),
        ("solver", ctypes.c_int),
        ("restart", ctypes.c_int),
        ("maxit", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("inner_steps", ctypes.c_int),
    ]


class FdeInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("inner_iters", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("relres_true", ctypes.c_double),
        ("relres_est", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FdeBatchCfg(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("grid", ctypes.c_int), ("lpt", ctypes.c_int), ("ms", ctypes.c_double),
                ("split", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FdeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Loads libfde.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1912_13304_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(FdeParams)
    lib.fde_default_params.argtypes = [dp]
    lib.fde_default_params.restype = None
    lib.fde_assemble.argtypes = [dp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.fde_assemble.restype = ctypes.c_int
    lib.fde_matvec.argtypes = [vp, vp, vp, vp]
    lib.fde_matvec.restype = ctypes.c_int
    lib.fde_tau_apply.argtypes = [vp, vp, vp, vp]
    lib.fde_tau_apply.restype = ctypes.c_int
    for name in ("fde_matvec_f32", "fde_tau_apply_f32"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
        getattr(lib, name).restype = ctypes.c_int
    lib.fde_solve.argtypes = [vp, vp, vp, ctypes.POINTER(FdeInfo), vp]
    lib.fde_solve.restype = ctypes.c_int
    lib.fde_rhs.argtypes = [vp, vp, vp, vp, vp]
    lib.fde_rhs.restype = ctypes.c_int
    lib.fde_plan_bytes.argtypes = [dp]
    lib.fde_plan_bytes.restype = ctypes.c_size_t
    lib.fde_destroy.argtypes = [vp]
    lib.fde_destroy.restype = None
    lib.fde_release_cache.argtypes = []
    lib.fde_release_cache.restype = None
    lib.fde_probe.argtypes = [vp, ctypes.c_int]
    lib.fde_probe.restype = ctypes.c_int
    lib.fde_probe_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(ctypes.c_double)]
    lib.fde_probe_read.restype = ctypes.c_int
    cp = ctypes.POINTER(FdeBatchCfg)
    lib.fde_batch_layout.argtypes = [dp, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
    lib.fde_batch_layout.restype = ctypes.c_size_t
    lib.fde_batch_bytes.argtypes = [dp, ctypes.c_int]
    lib.fde_batch_bytes.restype = ctypes.c_size_t
    lib.fde_batch_assemble.argtypes = [dp, ctypes.c_int, vp, vp, vp, ctypes.POINTER(vp)]
    lib.fde_batch_assemble.restype = ctypes.c_int
    lib.fde_batch_solve.argtypes = [vp, vp, vp, ctypes.POINTER(FdeInfo), vp]
    lib.fde_batch_solve.restype = ctypes.c_int
    lib.fde_batch_run.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(FdeInfo), vp]
    lib.fde_batch_run.restype = ctypes.c_int
    lib.fde_batch_tune.argtypes = [vp, vp, vp, cp]
    lib.fde_batch_tune.restype = ctypes.c_int
    lib.fde_batch_get_cfg.argtypes = [vp, cp]
    lib.fde_batch_get_cfg.restype = ctypes.c_int
    lib.fde_batch_set_cfg.argtypes = [vp, cp]
    lib.fde_batch_set_cfg.restype = ctypes.c_int
    lib.fde_batch_matvec.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.fde_batch_matvec.restype = ctypes.c_int
    lib.fde_batch_tau_apply.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.fde_batch_tau_apply.restype = ctypes.c_int
    lib.fde_batch_destroy.argtypes = [vp]
    lib.fde_batch_destroy.restype = None
    lib.fde_pcg1d_solve_noalloc.argtypes = [dp, vp, vp, vp, vp, ctypes.POINTER(FdeInfo), vp]
    lib.fde_pcg1d_solve_noalloc.restype = ctypes.c_int
    lib.fde_last_error.argtypes = []
    lib.fde_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def fde_last_error() -> str:
    return load().fde_last_error().decode()


def _check(status, allow_notconv=False):
    if status == FDE_OK or (allow_notconv and status == FDE_ENOTCONV):
        return status
    raise FdeError(status, fde_last_error())


def _ptr(t):
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("vectors must be contiguous float64 tensors on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def fde_default_params() -> FdeParams:
    p = FdeParams()
    load().fde_default_params(ctypes.byref(p))
    return p


def params_for(problem, **kw) -> FdeParams:
    """fde_params for a fde_inputs.Problem; keyword arguments override fields."""
    p = fde_default_params()
    p.dim = problem.dim
    p.n[0] = problem.n[0]
    p.n[1] = problem.n[1] if problem.dim == 2 else 1
    for i in range(problem.dim):
        p.alpha[i] = problem.alpha[i]
        p.lo[i] = problem.lo[i]
        p.hi[i] = problem.hi[i]
    p.dt = problem.dt
    p.weights = W_WEIGHTED if problem.weights == "weighted" else W_SHIFTED
    p.time = T_CN if problem.time == "cn" else T_EULER
    p.solver = S_PCG if problem.solver == "pcg" else S_GMRES
    p.restart = problem.restart
    p.tol = problem.tol
    for k, v in kw.items():
        if k in ("n", "alpha", "lo", "hi"):
            for i, x in enumerate(v):
                getattr(p, k)[i] = x
        else:
            setattr(p, k, v)
    return p


def fde_assemble(params: FdeParams, dplus, dminus, eplus=None, eminus=None, stream=None) -> ctypes.c_void_p:
    plan = ctypes.c_void_p()
    _check(load().fde_assemble(ctypes.byref(params), _ptr(dplus), _ptr(dminus), _ptr(eplus), _ptr(eminus),
                               _stream(stream), ctypes.byref(plan)))
    return plan


def fde_matvec(plan, x, y, stream=None):
    return _check(load().fde_matvec(plan, _ptr(x), _ptr(y), _stream(stream)))


def fde_tau_apply(plan, v, z, stream=None):
    return _check(load().fde_tau_apply(plan, _ptr(v), _ptr(z), _stream(stream)))


def fde_matvec_f32(plan, x, y, stream=None):
    return _check(load().fde_matvec_f32(plan, _ptr(x), _ptr(y), _stream(stream)))


def fde_tau_apply_f32(plan, v, z, stream=None):
    return _check(load().fde_tau_apply_f32(plan, _ptr(v), _ptr(z), _stream(stream)))


def fde_solve(plan, b, x, stream=None, allow_notconv=False) -> FdeInfo:
    info = FdeInfo()
    st = load().fde_solve(plan, _ptr(b), _ptr(x), ctypes.byref(info), _stream(stream))
    _check(st, allow_notconv)
    return info


def fde_pcg1d_solve_noalloc(params: FdeParams, dplus, dminus, b, x, stream=None, allow_notconv=False) -> FdeInfo:
    """The allocation-free one-shot 1D PCG solve (no plan)."""
    info = FdeInfo()
    st = load().fde_pcg1d_solve_noalloc(ctypes.byref(params), _ptr(dplus), _ptr(dminus), _ptr(b), _ptr(x),
                                        ctypes.byref(info), _stream(stream))
    _check(st, allow_notconv)
    return info


def fde_rhs(plan, u_prev, f, b, stream=None):
    return _check(load().fde_rhs(plan, _ptr(u_prev), _ptr(f), _ptr(b), _stream(stream)))


def fde_plan_bytes(params: FdeParams) -> int:
    return int(load().fde_plan_bytes(ctypes.byref(params)))


def fde_destroy(plan):
    if plan:
        load().fde_destroy(plan)


def fde_release_cache():
    load().fde_release_cache()


def fde_probe(plan, cls):
    return _check(load().fde_probe(plan, int(cls)))


def fde_probe_read(plan):
    """(milliseconds, launches, algorithmic bytes) accumulated since the last read."""
    ms, n, by = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
    _check(load().fde_probe_read(plan, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
    return ms.value, n.value, by.value


class Plan:
    """Owns an fde_plan built from a fde_inputs.Problem (coefficients copied to
    the GPU here)."""

    def __init__(self, problem, device="cuda", stream=None, **kw):
        import torch
        self.problem = problem
        self.params = params_for(problem, **kw)
        t = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64, device=device).contiguous()
        self._coef = [t(problem.dplus), t(problem.dminus), t(problem.eplus), t(problem.eminus)]
        self.handle = fde_assemble(self.params, *self._coef, stream=stream)
        self._coef = None

    def matvec(self, x, y, stream=None):
        fde_matvec(self.handle, x, y, stream)

    def tau_apply(self, v, z, stream=None):
        fde_tau_apply(self.handle, v, z, stream)

    def matvec_f32(self, x, y, stream=None):
        fde_matvec_f32(self.handle, x, y, stream)

    def tau_apply_f32(self, v, z, stream=None):
        fde_tau_apply_f32(self.handle, v, z, stream)

    def solve(self, b, x, stream=None, allow_notconv=False) -> FdeInfo:
        return fde_solve(self.handle, b, x, stream, allow_notconv)

    def rhs(self, u_prev, b, f=None, stream=None):
        fde_rhs(self.handle, u_prev, f, b, stream)

    def close(self):
        if self.handle:
            fde_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---------------------------------------------------------------------------
# Batched 1D solves (fde_batch_*)
# ---------------------------------------------------------------------------
def _params_array(params):
    arr = (FdeParams * len(params))()
    for i, p in enumerate(params):
        arr[i] = p
    return arr


def fde_batch_layout(params):
    """(offsets of the packed layout (count + 1 entries), total length)."""
    arr = _params_array(params)
    off = (ctypes.c_longlong * (len(params) + 1))()
    total = load().fde_batch_layout(arr, len(params), off)
    if total == 0:
        raise FdeError(FDE_EINVAL, fde_last_error())
    return list(off), int(total)


def fde_batch_bytes(params) -> int:
    arr = _params_array(params)
    return int(load().fde_batch_bytes(arr, len(params)))


class Batch:
    """Owns an fde_batch: many 1D instances (fde_inputs.Problem each) solved
    together.  Packed vectors are float64 CUDA tensors of length ``total``."""

    def __init__(self, problems, device="cuda", stream=None, **kw):
        import torch
        self.problems = list(problems)
        self.params = [params_for(p, **kw) for p in self.problems]
        self.offsets, self.total = fde_batch_layout(self.params)
        cat = lambda key: torch.as_tensor(
            [v for p in self.problems for v in list(getattr(p, key))], dtype=torch.float64, device=device)
        dp, dm = cat("dplus"), cat("dminus")
        arr = _params_array(self.params)
        h = ctypes.c_void_p()
        _check(load().fde_batch_assemble(arr, len(self.params), _ptr(dp), _ptr(dm), _stream(stream),
                                         ctypes.byref(h)))
        self.handle = h
        self.count = len(self.params)

    def pack(self, arrays, device="cuda"):
        import numpy as np
        import torch
        return torch.as_tensor(np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in arrays]),
                               dtype=torch.float64, device=device)

    def unpack(self, t):
        h = t.detach().cpu().numpy()
        return [h[self.offsets[i]:self.offsets[i + 1]] for i in range(self.count)]

    def solve(self, b, x, stream=None, allow_notconv=False):
        infos = (FdeInfo * self.count)()
        st = load().fde_batch_solve(self.handle, _ptr(b), _ptr(x), infos, _stream(stream))
        _check(st, allow_notconv)
        return list(infos)

    def run(self, u, steps, use_graph=True, stream=None, allow_notconv=False):
        """Advances the packed state u by `steps` implicit steps; returns
        infos[step][instance]."""
        infos = (FdeInfo * (steps * self.count))()
        st = load().fde_batch_run(self.handle, _ptr(u), int(steps), int(bool(use_graph)), infos, _stream(stream))
        _check(st, allow_notconv)
        return [list(infos[s * self.count:(s + 1) * self.count]) for s in range(steps)]

    def matvec(self, x, y, precision=FP64, stream=None):
        _check(load().fde_batch_matvec(self.handle, int(precision), _ptr(x), _ptr(y), _stream(stream)))

    def tau_apply(self, v, z, precision=FP64, stream=None):
        _check(load().fde_batch_tau_apply(self.handle, int(precision), _ptr(v), _ptr(z), _stream(stream)))

    def tune(self, u, stream=None) -> FdeBatchCfg:
        c = FdeBatchCfg()
        _check(load().fde_batch_tune(self.handle, _ptr(u), _stream(stream), ctypes.byref(c)))
        return c

    def get_cfg(self) -> FdeBatchCfg:
        c = FdeBatchCfg()
        _check(load().fde_batch_get_cfg(self.handle, ctypes.byref(c)))
        return c

    def set_cfg(self, variant, grid, lpt=1, split=0):
        c = FdeBatchCfg(int(variant), int(grid), int(lpt), 0.0, int(split))
        _check(load().fde_batch_set_cfg(self.handle, ctypes.byref(c)))

    def close(self):
        if getattr(self, "handle", None):
            load().fde_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
