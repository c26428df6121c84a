"""CPU FP64 oracle for the HODLR GP likelihood.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call, link or execute anything
under ``oracle/``.  The GPU product path shares no code with it and must never
route through it.

Contents
--------
* ``dense_oracle.c`` / ``gp_dense``: the plain definition -- dense
  C = sigma^2 I + K, Cholesky, log det, C^{-1} y and the log-likelihood
  (paper §1 Eq. (1), §2.1).
* ``kalman.c`` / ``kalman_matern32``: exact O(n) reference for 1-D Matern-3/2
  through the state-space form mentioned in §2.4.
* ``cross_matrix`` / ``gp_predict_dense``: the prediction of §2.1 (predictive
  mean and variance at new inputs) written out with dense matrices.
* ``matvec_rows``: exact rows of C v evaluated entry by entry, for residuals
  ||y - C x|| / ||y|| at sizes where C cannot be formed.
* ``hodlr_ref``: the method's own steps (tree, cross approximation, leaf
  factorization, level-by-level Sherman-Morrison-Woodbury, Sylvester
  determinant, solve) in numpy, for pinning intermediate quantities.
* ``mlp_ref``: the likelihood surrogate network (forward, gradient by the
  chain rule, Adam) in FP64 numpy.
* ``mcmc_ref``: plain and delayed-acceptance Metropolis decisions and an
  effective-sample-size estimator, for the sampler of the paper's outer loop.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["dense_oracle.c", "kalman.c"]
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O2, OpenMP, no fast-math)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-D_DEFAULT_SOURCE", *srcs, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.oracle_kernel.restype = ctypes.c_double
        L.oracle_kernel.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double]
        L.oracle_dense_matrix.restype = None
        L.oracle_dense_matrix.argtypes = [dp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, dp]
        L.oracle_cholesky.restype = ctypes.c_int
        L.oracle_cholesky.argtypes = [dp, i64]
        L.oracle_logdet_chol.restype = ctypes.c_double
        L.oracle_logdet_chol.argtypes = [dp, i64]
        L.oracle_chol_solve.restype = None
        L.oracle_chol_solve.argtypes = [dp, i64, dp, dp]
        L.oracle_gp.restype = ctypes.c_int
        L.oracle_gp.argtypes = [dp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, dp, dp, dp, dp, dp]
        L.oracle_cross_matrix.restype = None
        L.oracle_cross_matrix.argtypes = [dp, i64, dp, i64, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double, dp]
        L.oracle_matvec_rows.restype = None
        L.oracle_matvec_rows.argtypes = [dp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, dp,
                                         ctypes.POINTER(ctypes.c_int64), i64, dp]
        L.oracle_kalman_matern32.restype = ctypes.c_int
        L.oracle_kalman_matern32.argtypes = [dp, i64, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, dp, dp, dp, dp]
        L.oracle_kalman_matern32_noise.restype = ctypes.c_int
        L.oracle_kalman_matern32_noise.argtypes = [dp, i64, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_double, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pts(x):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    return x


class OracleError(RuntimeError):
    pass


def kernel_value(kind: int, xi, xj, a: float, ell: float) -> float:
    xi = np.ascontiguousarray(np.atleast_1d(np.asarray(xi, dtype=np.float64)))
    xj = np.ascontiguousarray(np.atleast_1d(np.asarray(xj, dtype=np.float64)))
    return lib().oracle_kernel(int(kind), _p(xi), _p(xj), int(xi.size), float(a), float(ell))


def dense_matrix(x, kind: int, theta, sigma2: float) -> np.ndarray:
    """C = sigma^2 I + K as a dense (n, n) float64 array."""
    x = _pts(x)
    n, dim = x.shape
    C = np.empty((n, n), dtype=np.float64)
    lib().oracle_dense_matrix(_p(x), n, dim, int(kind), float(theta[0]), float(theta[1]),
                              float(sigma2), _p(C))
    return C


def cholesky(C: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor of a dense SPD matrix (raises if not SPD)."""
    G = np.array(C, dtype=np.float64, order="C", copy=True)
    st = lib().oracle_cholesky(_p(G), G.shape[0])
    if st != 0:
        raise OracleError("matrix not positive definite (pivot %d)" % (st - 1))
    return G


def logdet_from_chol(G: np.ndarray) -> float:
    G = np.ascontiguousarray(G, dtype=np.float64)
    return lib().oracle_logdet_chol(_p(G), G.shape[0])


def chol_solve(G: np.ndarray, b) -> np.ndarray:
    G = np.ascontiguousarray(G, dtype=np.float64)
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).ravel())
    out = np.empty_like(b)
    lib().oracle_chol_solve(_p(G), G.shape[0], _p(b), _p(out))
    return out


def gp_dense(x, y, kind: int, theta, sigma2: float):
    """Plain definition: returns dict(logdet, quad, loglik, alpha=C^{-1}y)."""
    x = _pts(x)
    n, dim = x.shape
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).ravel())
    ld = ctypes.c_double()
    q = ctypes.c_double()
    ll = ctypes.c_double()
    alpha = np.empty(n, dtype=np.float64)
    st = lib().oracle_gp(_p(x), n, dim, int(kind), float(theta[0]), float(theta[1]),
                         float(sigma2), _p(y), ctypes.byref(ld), ctypes.byref(q),
                         ctypes.byref(ll), _p(alpha))
    if st == -1:
        raise MemoryError("oracle_gp: allocation failed for n=%d" % n)
    if st != 0:
        raise OracleError("covariance not positive definite (pivot %d)" % (st - 1))
    return {"logdet": ld.value, "quad": q.value, "loglik": ll.value, "alpha": alpha}


def gp_dense_noise(x, y, kind: int, theta, sigma2: float, noise):
    """§5's covariance C_ij = (sigma^2 + sigma_i^2) delta_ij + k(x_i, x_j) with
    per-point variances sigma_i^2 = noise[i] (caller's order), by the plain
    definitions: the oracle's dense K, the diagonal added, its Cholesky, log
    det = 2 sum log G_ii, alpha by the two triangular solves.  Returns the same
    dict as gp_dense."""
    x = _pts(x)
    n = x.shape[0]
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).ravel())
    noise = np.asarray(noise, dtype=np.float64).ravel()
    if noise.size != n:
        raise ValueError("noise must hold one variance per point")
    C = dense_matrix(x, kind, theta, sigma2)
    C[np.diag_indices(n)] += noise
    G = cholesky(C)
    ld = 2.0 * float(np.sum(np.log(np.diag(G))))
    alpha = chol_solve(G, y)
    q = float(y @ alpha)
    return {"logdet": ld, "quad": q, "loglik": -0.5 * q - 0.5 * ld - 0.5 * n * np.log(2.0 * np.pi),
            "alpha": alpha}


def cross_matrix(xa, xb, kind: int, theta) -> np.ndarray:
    """K(xa, xb) entry by entry (no noise term), shape (len(xa), len(xb))."""
    xa = _pts(xa)
    xb = _pts(xb)
    if xa.shape[1] != xb.shape[1]:
        raise ValueError("point sets of different dimension")
    out = np.empty((xa.shape[0], xb.shape[0]), dtype=np.float64)
    lib().oracle_cross_matrix(_p(xa), xa.shape[0], _p(xb), xb.shape[0], xa.shape[1], int(kind),
                              float(theta[0]), float(theta[1]), _p(out))
    return out


def gp_predict_dense(x, y, xt, kind: int, theta, sigma2: float, want_var: bool = True):
    """§2.1 prediction written out with dense FP64 matrices (mean function 0):
    mean = k(xt, x) C^{-1} y and var = k(xt, xt) - k(xt, x) C^{-1} k(x, xt), the
    variance of the latent f, with C = sigma^2 I + K factored by the oracle's
    Cholesky.  Returns (mean, var or None)."""
    C = dense_matrix(x, kind, theta, sigma2)
    G = cholesky(C)
    alpha = chol_solve(G, y)
    Ks = cross_matrix(xt, x, kind, theta)
    mean = Ks @ alpha
    if not want_var:
        return mean, None
    xt = _pts(xt)
    var = np.empty(xt.shape[0])
    for j in range(xt.shape[0]):
        v = chol_solve(G, Ks[j])
        var[j] = kernel_value(kind, xt[j], xt[j], theta[0], theta[1]) - Ks[j] @ v
    return mean, var


def matvec_rows(x, kind: int, theta, sigma2: float, v, rows) -> np.ndarray:
    """Rows ``rows`` of C v, with C evaluated entry by entry (O(n) per row)."""
    x = _pts(x)
    n, dim = x.shape
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).ravel())
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).ravel())
    out = np.empty(rows.size, dtype=np.float64)
    lib().oracle_matvec_rows(_p(x), n, dim, int(kind), float(theta[0]), float(theta[1]),
                             float(sigma2), _p(v),
                             rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             rows.size, _p(out))
    return out


def kalman_matern32(t, y, theta, sigma2: float, want_alpha: bool = True, noise=None):
    """Exact 1-D Matern-3/2 log det, quad and C^{-1}y in O(n) (t sorted);
    noise: optional per-point variances added to sigma2 (§5's sigma_i^2)."""
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64).ravel())
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).ravel())
    n = t.size
    ld = ctypes.c_double()
    q = ctypes.c_double()
    alpha = np.empty(n, dtype=np.float64) if want_alpha else None
    if noise is None:
        st = lib().oracle_kalman_matern32(_p(t), n, float(theta[0]), float(theta[1]),
                                          float(sigma2), _p(y), ctypes.byref(ld),
                                          ctypes.byref(q), _p(alpha) if want_alpha else None)
    else:
        nz = np.ascontiguousarray(np.asarray(noise, dtype=np.float64).ravel())
        if nz.size != n:
            raise ValueError("noise must hold one variance per point")
        st = lib().oracle_kalman_matern32_noise(_p(t), n, float(theta[0]), float(theta[1]),
                                                float(sigma2), _p(nz), _p(y), ctypes.byref(ld),
                                                ctypes.byref(q),
                                                _p(alpha) if want_alpha else None)
    if st != 0:
        raise OracleError("kalman oracle failed (status %d)" % st)
    loglik = -0.5 * q.value - 0.5 * ld.value - 0.5 * n * np.log(2.0 * np.pi)
    return {"logdet": ld.value, "quad": q.value, "loglik": loglik, "alpha": alpha}
