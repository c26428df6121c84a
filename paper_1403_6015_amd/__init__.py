"""MI355X HODLR Gaussian-process likelihoods: Python binding of libhodlrgp.

The names mirror the C ABI in ``include/hodlr.h``.  This module only marshals
arguments (numpy arrays for the host entry points, torch device tensors or
raw device pointers for the ``_dev`` entry points); every step of the
factorization, log-det and solve runs in the library's HIP kernels.  There
is no fallback: if the shared library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "HodlrError", "Opts", "Factor", "Plan", "lib", "hodlr_order", "hodlr_num_levels",
    "hodlr_build", "hodlr_logdet", "hodlr_solve", "hodlr_predict", "gp_loglik", "hodlr_info",
    "hodlr_free",
    "gp_loglik_dev", "hodlr_matvec_dev", "K_SE", "K_MATERN32", "K_EXP", "K_CONST", "K_IMQ",
    "FP64", "MIXED", "COMPRESS_ACA", "COMPRESS_SKETCH", "EXPORTED", "profile_enable", "profile_read", "gp_loglik_batch_dev",
    "gp_loglik_ragged", "MlpNorm", "SamplerCfg", "SamplerStats", "MLP_NPARAM",
    "mlp_workspace_size", "mlp_cast_dev", "mlp_forward_dev", "mlp_grad_dev", "mlp_train_step_dev",
    "mlp_train_step_noalloc_dev", "MLP_NOALLOC_MAX_BATCH", "mlp_fit_dev", "mh_propose_dev", "da_screen_dev", "da_accept_dev", "sampler_workspace_size",
    "gp_sample_dev", "Tune", "plan_tuned_create", "autotune", "tune_lookup", "gp_loglik_grad_dev",
]

K_SE, K_MATERN32, K_EXP, K_CONST, K_IMQ = 0, 1, 2, 3, 4
FP64, MIXED = 0, 1
COMPRESS_ACA, COMPRESS_SKETCH = 0, 1
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOTSPD", 3: "ENOMEM", 4: "EDEVICE", 5: "ENOCONV"}
EXPORTED = [
    "hodlr_order", "hodlr_num_levels", "hodlr_build", "hodlr_logdet", "hodlr_solve",
    "gp_loglik", "hodlr_info", "hodlr_free", "hodlr_last_error", "hodlr_plan_create",
    "hodlr_plan_destroy", "hodlr_plan_workspace_size", "gp_loglik_dev", "hodlr_matvec_dev",
    "hodlr_profile_enable", "hodlr_profile_read", "hodlr_plan_batch_workspace_size",
    "gp_loglik_batch_dev", "gp_loglik_ragged", "hodlr_mlp_workspace_size", "hodlr_mlp_cast_dev",
    "hodlr_mlp_forward_dev", "hodlr_mlp_grad_dev", "hodlr_mlp_train_step_dev",
    "hodlr_mlp_fit_dev", "hodlr_mh_propose_dev", "hodlr_da_screen_dev", "hodlr_da_accept_dev",
    "hodlr_sampler_workspace_size", "gp_sample_dev", "hodlr_plan_tuned_create", "hodlr_autotune",
    "hodlr_tune_lookup", "hodlr_profile_select", "hodlr_predict", "hodlr_mlp_train_step_noalloc_dev",
    "hodlr_plan_info", "hodlr_plan_grad_workspace_size", "gp_loglik_grad_dev",
]
MLP_NPARAM = 17153
MLP_NOALLOC_MAX_BATCH = 4096

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhodlrgp.so")
_lib = None
MAX_LEVELS = 40


class HodlrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status
        self.name = STATUS.get(status, str(status))


class Opts(ctypes.Structure):
    _fields_ = [("max_rank", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("presorted", ctypes.c_int32), ("noise", ctypes.c_void_p),
                ("refine", ctypes.c_int32), ("mixed_unchecked", ctypes.c_int32),
                ("compressor", ctypes.c_int32), ("speculate", ctypes.c_int32),
                ("level_form", ctypes.c_int32)]

    def __init__(self, max_rank=64, precision=FP64, refine_tol=1e-10, max_refine=8, presorted=0,
                 noise=None, refine=0, mixed_unchecked=0, compressor=0, speculate=0,
                 level_form=0):
        """noise: optional per-point variances (one per point, caller's order),
        added to sigma2 on the diagonal; the array is kept alive with the
        options."""
        self._noise = None
        ptr = None
        if noise is not None:
            self._noise = np.ascontiguousarray(np.asarray(noise, dtype=np.float64).ravel())
            ptr = self._noise.ctypes.data
        super().__init__(int(max_rank), int(precision), float(refine_tol), int(max_refine),
                         int(presorted), ptr, int(refine), int(mixed_unchecked), int(compressor),
                         int(speculate), int(level_form))


class Profile(ctypes.Structure):
    _fields_ = [("nstages", ctypes.c_int32), ("name", (ctypes.c_char * 32) * 16),
                ("ms", ctypes.c_double * 16), ("launches", ctypes.c_int64 * 16)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("leaf_max", ctypes.c_int32), ("max_rank_used", ctypes.c_int32),
                ("capped_blocks", ctypes.c_int32),
                ("rank_max", ctypes.c_int32 * MAX_LEVELS),
                ("rank_mean", ctypes.c_double * MAX_LEVELS),
                ("device_bytes", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("refine_residual", ctypes.c_double),
                ("fp64_fallback", ctypes.c_int32), ("speculated", ctypes.c_int32),
                ("projected", ctypes.c_int32)]


class MlpNorm(ctypes.Structure):
    _fields_ = [("mu_in", ctypes.c_float * 3), ("sd_in", ctypes.c_float * 3),
                ("mu_out", ctypes.c_float), ("sd_out", ctypes.c_float)]

    def __init__(self, mu_in=(0.0, 0.0, 0.0), sd_in=(1.0, 1.0, 1.0), mu_out=0.0, sd_out=1.0):
        super().__init__((ctypes.c_float * 3)(*mu_in), (ctypes.c_float * 3)(*sd_in),
                         float(mu_out), float(sd_out))

    def as_dict(self):
        return {"mu_in": [float(v) for v in self.mu_in], "sd_in": [float(v) for v in self.sd_in],
                "mu_out": float(self.mu_out), "sd_out": float(self.sd_out)}


class SamplerCfg(ctypes.Structure):
    _fields_ = [("walkers", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("chol", ctypes.c_double * 9), ("init_state", ctypes.c_int32)]

    def __init__(self, walkers, steps, lo, hi, chol, init_state=1):
        c = np.asarray(chol, dtype=np.float64).reshape(9)
        super().__init__(int(walkers), int(steps), (ctypes.c_double * 3)(*lo),
                         (ctypes.c_double * 3)(*hi), (ctypes.c_double * 9)(*c), int(init_state))


class Tune(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("level_rows", ctypes.c_int32),
                ("reduce_cols", ctypes.c_int32), ("reduce_group", ctypes.c_int32)]

    def __init__(self, leaf=128, level_rows=512, reduce_cols=4, reduce_group=8):
        super().__init__(int(leaf), int(level_rows), int(reduce_cols), int(reduce_group))

    def as_dict(self):
        return {"leaf": self.leaf, "level_rows": self.level_rows, "reduce_cols": self.reduce_cols,
                "reduce_group": self.reduce_group}


class SamplerStats(ctypes.Structure):
    _fields_ = [("proposals", ctypes.c_int64), ("survivors", ctypes.c_int64),
                ("exact_evals", ctypes.c_int64), ("accepted", ctypes.c_int64)]


def lib():
    """Load libhodlrgp.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhodlrgp.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7);
    # loading torch first makes this library bind to that runtime, so device
    # pointers and streams from torch are valid here and one process never
    # holds two HIP runtimes.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    st = ctypes.c_int
    L.hodlr_last_error.restype = ctypes.c_char_p
    L.hodlr_num_levels.restype = i32
    L.hodlr_num_levels.argtypes = [i64, i32]
    L.hodlr_order.restype = st
    L.hodlr_order.argtypes = [dp, i64, i32, i32, ctypes.POINTER(ctypes.c_int64)]
    L.hodlr_build.restype = st
    L.hodlr_build.argtypes = [dp, i64, i32, ctypes.c_int, dp, ctypes.c_double, i32,
                              ctypes.c_double, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.hodlr_logdet.restype = st
    L.hodlr_logdet.argtypes = [vp, dp]
    L.hodlr_solve.restype = st
    L.hodlr_solve.argtypes = [vp, dp, dp, i64]
    L.hodlr_predict.restype = st
    L.hodlr_predict.argtypes = [vp, dp, dp, i64, dp, dp]
    L.gp_loglik.restype = st
    L.gp_loglik.argtypes = [dp, i64, i32, ctypes.c_int, dp, ctypes.c_double, dp, i32,
                            ctypes.c_double, ctypes.POINTER(Opts), dp, dp, dp]
    L.hodlr_info.restype = st
    L.hodlr_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.hodlr_plan_info.restype = st
    L.hodlr_plan_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.hodlr_free.restype = None
    L.hodlr_free.argtypes = [vp]
    L.hodlr_plan_create.restype = st
    L.hodlr_plan_create.argtypes = [i64, i32, i32, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.hodlr_plan_destroy.restype = None
    L.hodlr_plan_destroy.argtypes = [vp]
    L.hodlr_plan_workspace_size.restype = st
    L.hodlr_plan_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.gp_loglik_dev.restype = st
    L.gp_loglik_dev.argtypes = [vp, vp, ctypes.c_int, dp, ctypes.c_double, vp, ctypes.c_double,
                                vp, ctypes.c_size_t, vp, vp, vp]
    L.hodlr_matvec_dev.restype = st
    L.hodlr_matvec_dev.argtypes = [i64, i32, vp, ctypes.c_int, dp, ctypes.c_double, vp, vp, vp]
    L.hodlr_plan_batch_workspace_size.restype = st
    L.hodlr_plan_batch_workspace_size.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.gp_loglik_batch_dev.restype = st
    L.gp_loglik_batch_dev.argtypes = [vp, vp, ctypes.c_int, vp, i32, vp, i64, ctypes.c_double, vp,
                                      ctypes.c_size_t, vp, vp, i32]
    L.hodlr_plan_grad_workspace_size.restype = st
    L.hodlr_plan_grad_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.gp_loglik_grad_dev.restype = st
    L.gp_loglik_grad_dev.argtypes = [vp, vp, ctypes.c_int, dp, ctypes.c_double, vp, ctypes.c_double,
                                     ctypes.c_double, vp, ctypes.c_size_t, vp, vp]
    L.gp_loglik_ragged.restype = st
    L.gp_loglik_ragged.argtypes = [i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(dp),
                                   ctypes.POINTER(dp), i32, ctypes.c_int, dp, i32, ctypes.c_double,
                                   ctypes.POINTER(Opts), i32, dp]
    fp = ctypes.POINTER(ctypes.c_float)
    szp = ctypes.POINTER(ctypes.c_size_t)
    nrm = ctypes.POINTER(MlpNorm)
    f32 = ctypes.c_float
    L.hodlr_mlp_workspace_size.restype = st
    L.hodlr_mlp_workspace_size.argtypes = [i32, szp]
    L.hodlr_mlp_cast_dev.restype = st
    L.hodlr_mlp_cast_dev.argtypes = [vp, vp, vp]
    L.hodlr_mlp_forward_dev.restype = st
    L.hodlr_mlp_forward_dev.argtypes = [vp, nrm, vp, i32, vp, vp]
    L.hodlr_mlp_grad_dev.restype = st
    L.hodlr_mlp_grad_dev.argtypes = [vp, nrm, vp, vp, i32, vp, ctypes.c_size_t, vp, vp, vp]
    L.hodlr_mlp_train_step_dev.restype = st
    L.hodlr_mlp_train_step_dev.argtypes = [vp, vp, vp, vp, i32, f32, nrm, vp, vp, vp, i32, vp,
                                           ctypes.c_size_t, vp, vp]
    L.hodlr_mlp_train_step_noalloc_dev.restype = st
    L.hodlr_mlp_train_step_noalloc_dev.argtypes = [vp, vp, vp, vp, i32, f32, nrm, vp, vp, vp, i32,
                                                   vp, vp]
    L.hodlr_mlp_fit_dev.restype = st
    L.hodlr_mlp_fit_dev.argtypes = [vp, vp, vp, vp, i32, f32, nrm, vp, vp, i32, vp, i32, i32, vp,
                                    ctypes.c_size_t, vp, vp]
    L.hodlr_mh_propose_dev.restype = st
    L.hodlr_mh_propose_dev.argtypes = [i32, vp, dp, vp, vp, vp]
    L.hodlr_da_screen_dev.restype = st
    L.hodlr_da_screen_dev.argtypes = [i32, vp, dp, dp, vp, vp, vp, vp, vp, vp, vp]
    L.hodlr_da_accept_dev.restype = st
    L.hodlr_da_accept_dev.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.hodlr_sampler_workspace_size.restype = st
    L.hodlr_sampler_workspace_size.argtypes = [vp, i32, szp]
    L.gp_sample_dev.restype = st
    L.gp_sample_dev.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_double, vp, nrm,
                                ctypes.POINTER(SamplerCfg), vp, vp, vp, vp, vp, vp, vp,
                                ctypes.c_size_t, vp, vp, ctypes.POINTER(SamplerStats)]
    del fp
    L.hodlr_plan_tuned_create.restype = st
    L.hodlr_plan_tuned_create.argtypes = [i64, i32, ctypes.POINTER(Opts), ctypes.POINTER(Tune),
                                          ctypes.POINTER(vp)]
    L.hodlr_autotune.restype = st
    L.hodlr_autotune.argtypes = [dp, i64, i32, ctypes.c_int, dp, ctypes.c_double, dp,
                                 ctypes.c_double, ctypes.POINTER(Opts),
                                 ctypes.POINTER(ctypes.c_int32), i32, i32, ctypes.POINTER(Tune), dp]
    L.hodlr_tune_lookup.restype = st
    L.hodlr_tune_lookup.argtypes = [i64, i32, ctypes.c_int, i32, ctypes.POINTER(Tune)]
    L.hodlr_profile_select.restype = st
    L.hodlr_profile_select.argtypes = [ctypes.c_uint32]
    L.hodlr_profile_enable.restype = st
    L.hodlr_profile_enable.argtypes = [i32]
    L.hodlr_profile_read.restype = st
    L.hodlr_profile_read.argtypes = [ctypes.POINTER(Profile)]
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise HodlrError(status, lib().hodlr_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pts(x):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    return x


def _theta(theta):
    return np.ascontiguousarray(np.asarray(theta, dtype=np.float64).ravel()[:2])


def _ptr(t):
    """Device pointer of a torch tensor (or an int address); None -> NULL."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def hodlr_num_levels(n: int, leaf: int) -> int:
    return int(lib().hodlr_num_levels(int(n), int(leaf)))


def hodlr_order(x, leaf: int) -> np.ndarray:
    x = _pts(x)
    n, dim = x.shape
    perm = np.empty(n, dtype=np.int64)
    _check(lib().hodlr_order(_dp(x), n, dim, int(leaf),
                             perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return perm


class Factor:
    """Owning handle of a library factor (hodlr_build ... hodlr_free)."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        if not self._h:
            raise HodlrError(1, "factor already freed")
        return self._h

    def logdet(self) -> float:
        return hodlr_logdet(self)

    def solve(self, y) -> np.ndarray:
        return hodlr_solve(self, y)

    def predict(self, y, xt, var: bool = True):
        return hodlr_predict(self, y, xt, var)

    def info(self) -> dict:
        return hodlr_info(self)

    def free(self):
        if self._h:
            lib().hodlr_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _noise_len(opts, n):
    if opts is not None and opts._noise is not None and opts._noise.size != n:
        raise ValueError("opts.noise must hold one variance per point (%d, got %d)"
                         % (n, opts._noise.size))


def hodlr_build(x, kernel: int, theta, sigma2: float, leaf: int, tol: float,
                opts: Opts | None = None) -> Factor:
    x = _pts(x)
    n, dim = x.shape
    _noise_len(opts, n)
    th = _theta(theta)
    h = ctypes.c_void_p()
    _check(lib().hodlr_build(_dp(x), n, dim, int(kernel), _dp(th), float(sigma2), int(leaf),
                             float(tol), ctypes.byref(opts) if opts is not None else None,
                             ctypes.byref(h)))
    return Factor(h.value)


def hodlr_logdet(f: Factor) -> float:
    out = ctypes.c_double()
    _check(lib().hodlr_logdet(f.handle, ctypes.byref(out)))
    return out.value


def hodlr_predict(f: Factor, y, xt, var: bool = True):
    """Predictive mean (and variance of f, if var) at the rows of xt (§2.1):
    returns (mean, var or None) as float64 arrays of len(xt)."""
    info = hodlr_info(f)
    Y = np.ascontiguousarray(y, dtype=np.float64).ravel()
    if Y.size != info["n"]:
        raise HodlrError(1, "y must hold the factor's n observations")
    XT = np.asarray(xt, dtype=np.float64)
    if XT.ndim == 1:
        XT = XT.reshape(-1, 1)
    XT = np.ascontiguousarray(XT)
    if XT.ndim != 2 or XT.shape[1] != info["dim"]:
        raise HodlrError(1, "xt must be m x dim with the factor's dim")
    m = XT.shape[0]
    mean = np.empty(m)
    v = np.empty(m) if var else None
    _check(lib().hodlr_predict(f.handle, _dp(Y), _dp(XT), m, _dp(mean),
                               _dp(v) if v is not None else None))
    return mean, v


def hodlr_solve(f: Factor, y) -> np.ndarray:
    y = np.asarray(y, dtype=np.float64)
    vec = y.ndim == 1
    Y = np.asfortranarray(y.reshape(y.shape[0], -1))
    X = np.empty_like(Y, order="F")
    _check(lib().hodlr_solve(f.handle, _dp(Y), _dp(X), Y.shape[1]))
    return X[:, 0].copy() if vec else X


def gp_loglik(x, y, kernel: int, theta, sigma2: float, leaf: int, tol: float,
              opts: Opts | None = None):
    """Returns (loglik, logdet, quad)."""
    x = _pts(x)
    n, dim = x.shape
    _noise_len(opts, n)
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).ravel())
    th = _theta(theta)
    ll, ld, q = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().gp_loglik(_dp(x), n, dim, int(kernel), _dp(th), float(sigma2), _dp(y),
                           int(leaf), float(tol),
                           ctypes.byref(opts) if opts is not None else None,
                           ctypes.byref(ll), ctypes.byref(ld), ctypes.byref(q)))
    return ll.value, ld.value, q.value


def _info_dict(I) -> dict:
    L = I.levels
    return {"n": I.n, "dim": I.dim, "levels": L, "leaf_max": I.leaf_max,
            "max_rank_used": I.max_rank_used, "capped_blocks": I.capped_blocks,
            "rank_max": list(I.rank_max[:L]), "rank_mean": list(I.rank_mean[:L]),
            "device_bytes": I.device_bytes, "precision": I.precision,
            "refine_steps": I.refine_steps, "refine_residual": I.refine_residual,
            "fp64_fallback": I.fp64_fallback, "speculated": I.speculated,
            "projected": I.projected}


def hodlr_info(f: Factor) -> dict:
    I = Info()
    _check(lib().hodlr_info(f.handle, ctypes.byref(I)))
    return _info_dict(I)


def hodlr_free(f: Factor):
    f.free()


class Plan:
    """hodlr_plan_create (or hodlr_plan_tuned_create when ``tune`` is given) /
    hodlr_plan_workspace_size / hodlr_plan_destroy."""

    def __init__(self, n: int, dim: int, leaf: int, opts: Opts | None = None,
                 tune: "Tune | None" = None):
        h = ctypes.c_void_p()
        if tune is not None:
            leaf = tune.leaf
            _check(lib().hodlr_plan_tuned_create(int(n), int(dim),
                                                 ctypes.byref(opts) if opts is not None else None,
                                                 ctypes.byref(tune), ctypes.byref(h)))
        else:
            _check(lib().hodlr_plan_create(int(n), int(dim), int(leaf),
                                           ctypes.byref(opts) if opts is not None else None,
                                           ctypes.byref(h)))
        self._h = h.value
        self.n, self.dim, self.leaf = int(n), int(dim), int(leaf)
        sz = ctypes.c_size_t()
        _check(lib().hodlr_plan_workspace_size(self._h, ctypes.byref(sz)))
        self.workspace_bytes = int(sz.value)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        """hodlr_plan_info: the tree and the ranks of the last completed
        gp_loglik_dev call on this plan."""
        I = Info()
        _check(lib().hodlr_plan_info(self._h, ctypes.byref(I)))
        return _info_dict(I)

    def batch_workspace_bytes(self, nitems: int) -> int:
        sz = ctypes.c_size_t()
        _check(lib().hodlr_plan_batch_workspace_size(self._h, int(nitems), ctypes.byref(sz)))
        return int(sz.value)

    @property
    def grad_workspace_bytes(self) -> int:
        sz = ctypes.c_size_t()
        _check(lib().hodlr_plan_grad_workspace_size(self._h, ctypes.byref(sz)))
        return int(sz.value)

    def destroy(self):
        if self._h:
            lib().hodlr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def gp_loglik_dev(plan: Plan, d_x, kernel: int, theta, sigma2: float, d_y, tol: float, work,
                  work_bytes: int, stream, d_out, d_z=None):
    """Device entry point; d_x / d_y / work / d_out / d_z are torch device
    tensors (or raw addresses); stream is a torch stream, a raw handle, or None."""
    th = _theta(theta)
    s = None if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
    _check(lib().gp_loglik_dev(plan.handle, _ptr(d_x), int(kernel), _dp(th), float(sigma2),
                               _ptr(d_y), float(tol), _ptr(work), int(work_bytes), s,
                               _ptr(d_out), _ptr(d_z)))


def gp_loglik_batch_dev(plan: Plan, d_x, kernel: int, d_params, nitems: int, d_y, y_stride: int,
                        tol: float, work, work_bytes: int, stream, d_out, use_graph: bool = True):
    """Batched device entry point: d_params is an (nitems, 3) device tensor of
    (a, l, sigma^2); d_out receives (nitems, 3) {loglik, logdet, quad}."""
    s = None if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
    _check(lib().gp_loglik_batch_dev(plan.handle, _ptr(d_x), int(kernel), _ptr(d_params),
                                     int(nitems), _ptr(d_y), int(y_stride), float(tol), _ptr(work),
                                     int(work_bytes), s, _ptr(d_out), 1 if use_graph else 0))


def gp_loglik_grad_dev(plan: Plan, d_x, kernel: int, theta, sigma2: float, d_y, tol: float,
                       rel_step: float, work, work_bytes: int, stream, d_out):
    """Log-likelihood and its gradient in (a, l, sigma^2) by central
    differences over one batched call; d_out (device, 6 doubles) receives
    {loglik, logdet, quad, dL/da, dL/dl, dL/dsigma2}.  rel_step <= 0 takes
    the library's default."""
    th = _theta(theta)
    s = None if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
    _check(lib().gp_loglik_grad_dev(plan.handle, _ptr(d_x), int(kernel), _dp(th), float(sigma2),
                                    _ptr(d_y), float(tol), float(rel_step), _ptr(work),
                                    int(work_bytes), s, _ptr(d_out)))


def gp_loglik_ragged(xs, ys, kernel: int, params, leaf: int, tol: float,
                     opts: Opts | None = None, nworkers: int = 8) -> np.ndarray:
    """Log-likelihoods of independent problems of uneven size (host arrays).
    xs[i]: (n_i, dim) or (n_i,) points; ys[i]: n_i observations; params:
    (m, 3) rows (a, l, sigma^2).  Returns (m, 3) {loglik, logdet, quad}; NaN
    rows mark items that failed."""
    m = len(xs)
    if len(ys) != m:
        raise ValueError("xs and ys differ in length")
    X = [_pts(x) for x in xs]
    dim = X[0].shape[1] if m else 1
    if any(x.shape[1] != dim for x in X):
        raise ValueError("all items must share dim")
    Y = [np.ascontiguousarray(np.asarray(y, dtype=np.float64).ravel()) for y in ys]
    ns = np.array([x.shape[0] for x in X], dtype=np.int64)
    P = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(m, 3))
    dpt = ctypes.POINTER(ctypes.c_double)
    xa = (dpt * m)(*[_dp(x) for x in X])
    ya = (dpt * m)(*[_dp(y) for y in Y])
    out = np.empty((m, 3), dtype=np.float64)
    _check(lib().gp_loglik_ragged(m, ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), xa, ya,
                                  int(dim), int(kernel), _dp(P), int(leaf), float(tol),
                                  ctypes.byref(opts) if opts is not None else None,
                                  int(nworkers), _dp(out)))
    return out


def _stream(stream):
    return None if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)


def _host3(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).ravel())


def mlp_workspace_size(batch: int) -> int:
    sz = ctypes.c_size_t()
    _check(lib().hodlr_mlp_workspace_size(int(batch), ctypes.byref(sz)))
    return int(sz.value)


def mlp_cast_dev(d_master, d_wbf16, stream=None):
    _check(lib().hodlr_mlp_cast_dev(_ptr(d_master), _ptr(d_wbf16), _stream(stream)))


def mlp_forward_dev(d_wbf16, norm: MlpNorm, d_logtheta, batch: int, d_out, stream=None):
    _check(lib().hodlr_mlp_forward_dev(_ptr(d_wbf16), ctypes.byref(norm), _ptr(d_logtheta),
                                       int(batch), _ptr(d_out), _stream(stream)))


def mlp_grad_dev(d_wbf16, norm: MlpNorm, d_logtheta, d_target, batch: int, work, work_bytes: int,
                 d_grad, d_loss=None, stream=None):
    _check(lib().hodlr_mlp_grad_dev(_ptr(d_wbf16), ctypes.byref(norm), _ptr(d_logtheta),
                                    _ptr(d_target), int(batch), _ptr(work), int(work_bytes),
                                    _ptr(d_grad), _ptr(d_loss), _stream(stream)))


def mlp_train_step_dev(d_master, d_wbf16, d_m, d_v, step: int, lr: float, norm: MlpNorm,
                       d_logtheta, d_target, batch: int, work, work_bytes: int, d_loss=None,
                       stream=None, d_index=None):
    _check(lib().hodlr_mlp_train_step_dev(_ptr(d_master), _ptr(d_wbf16), _ptr(d_m), _ptr(d_v),
                                          int(step), float(lr), ctypes.byref(norm),
                                          _ptr(d_logtheta), _ptr(d_target), _ptr(d_index),
                                          int(batch), _ptr(work), int(work_bytes), _ptr(d_loss),
                                          _stream(stream)))


def mlp_train_step_noalloc_dev(d_master, d_wbf16, d_m, d_v, step: int, lr: float, norm: MlpNorm,
                               d_logtheta, d_target, batch: int, d_loss=None, stream=None,
                               d_index=None):
    _check(lib().hodlr_mlp_train_step_noalloc_dev(_ptr(d_master), _ptr(d_wbf16), _ptr(d_m),
                                                  _ptr(d_v), int(step), float(lr),
                                                  ctypes.byref(norm), _ptr(d_logtheta),
                                                  _ptr(d_target), _ptr(d_index), int(batch),
                                                  _ptr(d_loss), _stream(stream)))


def mlp_fit_dev(d_master, d_wbf16, d_m, d_v, step0: int, lr: float, norm: MlpNorm, d_logtheta,
                d_target, n: int, d_perm, epochs: int, batch: int, work, work_bytes: int,
                d_loss_hist=None, stream=None):
    _check(lib().hodlr_mlp_fit_dev(_ptr(d_master), _ptr(d_wbf16), _ptr(d_m), _ptr(d_v),
                                   int(step0), float(lr), ctypes.byref(norm), _ptr(d_logtheta),
                                   _ptr(d_target), int(n), _ptr(d_perm), int(epochs), int(batch),
                                   _ptr(work), int(work_bytes), _ptr(d_loss_hist),
                                   _stream(stream)))


def mh_propose_dev(w: int, d_theta, chol, d_eps, d_prop, stream=None):
    c = _host3(chol)
    _check(lib().hodlr_mh_propose_dev(int(w), _ptr(d_theta), _dp(c), _ptr(d_eps), _ptr(d_prop),
                                      _stream(stream)))


def da_screen_dev(w: int, d_prop, lo, hi, d_sur, d_sur_prop, d_u1, d_slot, d_count, d_params,
                  stream=None):
    lo, hi = _host3(lo), _host3(hi)
    _check(lib().hodlr_da_screen_dev(int(w), _ptr(d_prop), _dp(lo), _dp(hi), _ptr(d_sur),
                                     _ptr(d_sur_prop), _ptr(d_u1), _ptr(d_slot), _ptr(d_count),
                                     _ptr(d_params), _stream(stream)))


def da_accept_dev(w: int, delayed: bool, d_slot, d_exact, d_u, d_prop, d_sur_prop, d_theta, d_lp,
                  d_sur, d_accepted=None, stream=None):
    _check(lib().hodlr_da_accept_dev(int(w), 1 if delayed else 0, _ptr(d_slot), _ptr(d_exact),
                                     _ptr(d_u), _ptr(d_prop), _ptr(d_sur_prop), _ptr(d_theta),
                                     _ptr(d_lp), _ptr(d_sur), _ptr(d_accepted), _stream(stream)))


def sampler_workspace_size(plan: Plan, walkers: int) -> int:
    sz = ctypes.c_size_t()
    _check(lib().hodlr_sampler_workspace_size(plan.handle, int(walkers), ctypes.byref(sz)))
    return int(sz.value)


def gp_sample_dev(plan: Plan, d_x, kernel: int, d_y, tol: float, d_wbf16, norm, cfg: SamplerCfg,
                  d_theta, d_lp, d_sur, d_eps, d_u1, d_u2, work, work_bytes: int, stream=None,
                  d_chain=None) -> dict:
    """Runs cfg.steps sampler steps (delayed form if d_wbf16 is given);
    returns the tallies {proposals, survivors, exact_evals, accepted}."""
    S = SamplerStats()
    _check(lib().gp_sample_dev(plan.handle, _ptr(d_x), int(kernel), _ptr(d_y), float(tol),
                               _ptr(d_wbf16), ctypes.byref(norm) if norm is not None else None,
                               ctypes.byref(cfg), _ptr(d_theta), _ptr(d_lp), _ptr(d_sur),
                               _ptr(d_eps), _ptr(d_u1), _ptr(d_u2), _ptr(work), int(work_bytes),
                               _stream(stream), _ptr(d_chain), ctypes.byref(S)))
    return {"proposals": S.proposals, "survivors": S.survivors, "exact_evals": S.exact_evals,
            "accepted": S.accepted}


def plan_tuned_create(n: int, dim: int, tune: Tune, opts: Opts | None = None) -> Plan:
    return Plan(n, dim, tune.leaf, opts, tune)


def autotune(x, y, kernel: int, theta, sigma2: float, tol: float, opts: Opts | None = None,
             leaf_cands=None, reps: int = 3):
    """Returns (Tune, per-candidate ms list) from hodlr_autotune."""
    x = _pts(x)
    n, dim = x.shape
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).ravel())
    th = _theta(theta)
    lc = None if leaf_cands is None else np.ascontiguousarray(leaf_cands, dtype=np.int32)
    nl = 0 if lc is None else len(lc)
    times = np.zeros((nl if nl else 4) + 12)
    best = Tune()
    _check(lib().hodlr_autotune(_dp(x), n, dim, int(kernel), _dp(th), float(sigma2), _dp(y),
                                float(tol), ctypes.byref(opts) if opts is not None else None,
                                None if lc is None else lc.ctypes.data_as(
                                    ctypes.POINTER(ctypes.c_int32)),
                                nl, int(reps), ctypes.byref(best), _dp(times)))
    return best, times.tolist()


def tune_lookup(n: int, dim: int, kernel: int, precision: int = FP64) -> Tune:
    t = Tune()
    _check(lib().hodlr_tune_lookup(int(n), int(dim), int(kernel), int(precision), ctypes.byref(t)))
    return t


def hodlr_matvec_dev(n: int, dim: int, d_x, kernel: int, theta, sigma2: float, d_v, d_out,
                     stream=None):
    th = _theta(theta)
    s = None if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
    _check(lib().hodlr_matvec_dev(int(n), int(dim), _ptr(d_x), int(kernel), _dp(th),
                                  float(sigma2), _ptr(d_v), _ptr(d_out), s))


def profile_enable(on: bool = True):
    """Start (and reset) or stop per-kernel HIP-event timing inside the library."""
    _check(lib().hodlr_profile_enable(1 if on else 0))


PROFILE_STAGES = ["aca_row_pass", "aca_col_pass", "aca_small", "aca_misc", "leaf_factor",
                  "leaf_solve", "level_reduce", "level_solve", "level_update", "finish", "matvec",
                  "predict"]


def profile_select(stages=None):
    """Time only the named kernel kinds (None: all)."""
    mask = 0xFFFFFFFF if stages is None else sum(1 << PROFILE_STAGES.index(s) for s in stages)
    _check(lib().hodlr_profile_select(mask))


def profile_read() -> dict:
    """{kernel kind: (summed ms, launches)} for completed calls since the reset."""
    P = Profile()
    _check(lib().hodlr_profile_read(ctypes.byref(P)))
    return {P.name[i].value.decode(): (P.ms[i], int(P.launches[i])) for i in range(P.nstages)}
