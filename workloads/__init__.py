"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers (numpy PCG64 via ``default_rng``) and
arranges them into arrays.  It holds none of the factorization's arithmetic,
so both the CPU oracle and the GPU path can be fed byte-identical inputs
from it without sharing any code of the method.

The paper measures only on uniformly random synthetic points (§5, the
Gaussian/exponential tables: points drawn uniformly in a box) and on a
synthetic regression model (§5.6).  The configurations below keep that
recipe and the sizes of the workloads this library is benchmarked on:

* ``se1d_small``    n = 2048, x ~ U(-1, 1) sorted, SE kernel a=1, l=0.1,
                    sigma^2 = 0.01, leaf 64, tol 1e-12.
* ``matern1d``      n = 2^20, t ~ U(0, 1000) sorted, Matern-3/2 a=1, l=5,
                    sigma^2 = 0.1, leaf 128, tol 1e-10 (and density-matched
                    slices of it at smaller n for parity runs).
* ``se2d``          n = 2^22 points ~ U([0,1]^2), SE l=0.05,
                    sigma^2 = 1e-2, leaf 256, rank cap 64.
* ``batched_theta`` 256 hyperparameter triples on one shared 1-D x,
                    n = 65536; ``batched_ragged`` 512 independent series with
                    n log-uniform in [1024, 131072].
* ``learned``       n = 2^18 time series drawn from a Matern-3/2 GP.
* ``regression_model``  the synthetic regression model of §5.6: 1024 points
                    x ~ U(-3, 3), y = sin(2x) + exp(x)/8 + N(0, 1) noise, SE
                    kernel exp(-(x - x')^2), sigma^2 = 1, leaf 20.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# kernel identifiers (same numbering as the C-ABI enum hodlr_kernel)
K_SE = 0
K_MATERN32 = 1
K_EXP = 2
K_CONST = 3
K_IMQ = 4
KERNEL_NAMES = {K_SE: "se", K_MATERN32: "matern32", K_EXP: "exp", K_CONST: "const",
                K_IMQ: "imq"}


@dataclass
class GPProblem:
    """One GP likelihood problem: points, observations and hyperparameters."""
    name: str
    x: np.ndarray            # (n, dim) float64, caller order (1-D inputs are sorted)
    y: np.ndarray            # (n,) float64
    kernel: int
    theta: tuple             # (a, ell)
    sigma2: float
    leaf: int
    tol: float
    max_rank: int = 0        # 0 = library default
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def dim(self) -> int:
        return int(self.x.shape[1])


def _sorted_uniform(rng, lo, hi, n):
    return np.sort(rng.uniform(lo, hi, size=n)).astype(np.float64).reshape(n, 1)


def se1d_small(n: int = 2048) -> GPProblem:
    """n points U(-1,1) sorted (seed 101); y ~ N(0,1) (seed 201); SE a=1, l=0.1."""
    x = _sorted_uniform(np.random.default_rng(101), -1.0, 1.0, n)
    y = np.random.default_rng(201).standard_normal(n)
    return GPProblem("se1d_n%d" % n, x, y, K_SE, (1.0, 0.1), 0.01, 64, 1e-12)


def matern1d(n: int = 1 << 20, span: float | None = None) -> GPProblem:
    """Matern-3/2 time series, t ~ U(0, span) sorted (seed 102), y ~ N(0,1) (seed 202).

    The full workload is n = 2^20 on a span of 1000 (about 1049 points per
    unit, about 5200 per length scale).  With ``span=None`` a smaller n keeps
    that point density (span = 1000 * n / 2^20), so the off-diagonal ranks and
    the conditioning match the full-size problem.
    """
    if span is None:
        span = 1000.0 * n / float(1 << 20)
    x = _sorted_uniform(np.random.default_rng(102), 0.0, span, n)
    y = np.random.default_rng(202).standard_normal(n)
    return GPProblem("matern1d_n%d" % n, x, y, K_MATERN32, (1.0, 5.0), 0.1, 128, 1e-10,
                     meta={"span": span})


def clustered1d(n: int = 4096, kernel: int = K_MATERN32, seed: int = 103) -> GPProblem:
    """Half the points ~ U(0, 1), half ~ U(100, 1000), sorted; y ~ N(0,1).

    With l = 0.1 the leaves of the dense half span about c * 0.06 in units of
    the kernel's decay, those of the sparse half thousands, so one problem has
    leaves of both kinds for kernels whose leaf evaluation depends on the span.
    """
    rng = np.random.default_rng(seed)
    h = n // 2
    x = np.sort(np.concatenate([rng.uniform(0.0, 1.0, h), rng.uniform(100.0, 1000.0, n - h)]))
    y = np.random.default_rng(seed + 100).standard_normal(n)
    return GPProblem("clustered1d_n%d_k%d" % (n, kernel), x.astype(np.float64).reshape(n, 1), y,
                     kernel, (1.0, 0.1), 0.05, 128, 1e-12)


def se2d(n: int = 1 << 22, side: float | None = None, max_rank: int = 64) -> GPProblem:
    """2-D points ~ U([0,side]^2) (seed 103), y ~ N(0,1) (seed 203), SE l=0.05.

    The full workload is n = 2^22 on the unit square; ``side=None`` with a
    smaller n keeps the same density (side = sqrt(n / 2^22)).  The library
    orders the points by a count-median k-d split.
    """
    if side is None:
        side = math.sqrt(n / float(1 << 22))
    x = np.random.default_rng(103).uniform(0.0, side, size=(n, 2)).astype(np.float64)
    y = np.random.default_rng(203).standard_normal(n)
    return GPProblem("se2d_n%d" % n, x, y, K_SE, (1.0, 0.05), 1e-2, 256, 1e-10,
                     max_rank=max_rank, meta={"side": side})


def theta_box(m: int, seed: int = 104):
    """m hyperparameter triples, each log-uniform: a in [0.1,10], l in [0.01,1],
    sigma^2 in [1e-3, 1].  Returns an (m, 3) float64 array (a, l, sigma^2)."""
    rng = np.random.default_rng(seed)
    lo = np.log([0.1, 0.01, 1e-3])
    hi = np.log([10.0, 1.0, 1.0])
    return np.exp(rng.uniform(lo, hi, size=(m, 3)))


def batched_theta(m: int = 256, n: int = 65536):
    """Shared sorted x ~ U(0,10) (seed 104) with y ~ N(0,1) (seed 204), and m
    hyperparameter triples from ``theta_box`` (seed 105)."""
    x = _sorted_uniform(np.random.default_rng(104), 0.0, 10.0, n)
    y = np.random.default_rng(204).standard_normal(n)
    return x, y, theta_box(m, seed=105)


def batched_ragged(m: int = 512, nmin: int = 1024, nmax: int = 131072, seed0: int = 10000):
    """m independent 1-D series; n_i log-uniform in [nmin, nmax] (seed 106),
    x_i ~ U(0,10) sorted and y_i ~ N(0,1) from seed seed0+i, theta_i from
    ``theta_box`` (seed 107).  Returns (list of x, list of y, thetas)."""
    ns = np.rint(np.exp(np.random.default_rng(106).uniform(
        np.log(nmin), np.log(nmax), size=m))).astype(np.int64)
    xs, ys = [], []
    for i, ni in enumerate(ns):
        rng = np.random.default_rng(seed0 + i)
        xs.append(np.sort(rng.uniform(0.0, 10.0, size=int(ni))).reshape(-1, 1))
        ys.append(rng.standard_normal(int(ni)))
    return xs, ys, theta_box(m, seed=107)


def matern32_path(t: np.ndarray, a: float, ell: float, sigma2: float, seed: int) -> np.ndarray:
    """Exact draw y = f(t) + noise with f ~ GP(0, Matern-3/2(a, ell)) at sorted t.

    The Matern-3/2 process is the first component of a two-dimensional linear
    SDE (the state-space view of stationary kernels in §2.4 of the paper), so
    a draw at sorted times is a Markov chain: s_i = A(dt) s_{i-1} + q_i with
    q_i ~ N(0, P_inf - A P_inf A^T).  This is data generation only; no
    likelihood arithmetic lives here.
    """
    rng = np.random.default_rng(seed)
    t = np.asarray(t, dtype=np.float64).ravel()
    n = t.size
    lam = math.sqrt(3.0) / ell
    pinf = np.diag([a * a, lam * lam * a * a])
    s = np.linalg.cholesky(pinf) @ rng.standard_normal(2)
    f = np.empty(n)
    f[0] = s[0]
    z = rng.standard_normal((n, 2))
    for i in range(1, n):
        dt = t[i] - t[i - 1]
        e = math.exp(-lam * dt)
        A = e * np.array([[1.0 + lam * dt, dt], [-lam * lam * dt, 1.0 - lam * dt]])
        Q = pinf - A @ pinf @ A.T
        Q = 0.5 * (Q + Q.T)
        w, V = np.linalg.eigh(Q)
        w = np.clip(w, 0.0, None)
        s = A @ s + V @ (np.sqrt(w) * z[i])
        f[i] = s[0]
    return f + math.sqrt(sigma2) * np.random.default_rng(seed + 1).standard_normal(n)


def learned(n: int = 1 << 18, theta_true=(1.0, 5.0, 0.1)) -> GPProblem:
    """Time series for the surrogate-screened sampler: t ~ U(0,1000) sorted
    (seed 108), y drawn from GP(0, Matern-3/2(a, l) + sigma^2 I) at theta_true."""
    t = _sorted_uniform(np.random.default_rng(108), 0.0, 1000.0, n)
    a, ell, s2 = theta_true
    y = matern32_path(t, a, ell, s2, seed=208)
    return GPProblem("learned_n%d" % n, t, y, K_MATERN32, (a, ell), s2, 128, 1e-10,
                     meta={"theta_true": tuple(theta_true)})


def rank1_points(n: int, seed: int = 7) -> GPProblem:
    """Small 1-D problem for the constant (rank-1) kernel pins."""
    x = _sorted_uniform(np.random.default_rng(seed), -1.0, 1.0, n)
    y = np.random.default_rng(seed + 1).standard_normal(n)
    return GPProblem("const_n%d" % n, x, y, K_CONST, (0.7, 1.0), 0.3, 16, 1e-12)


def random_problem(n: int, dim: int, kernel: int, seed: int, a: float = 1.0, ell: float = 0.3,
                   sigma2: float = 0.05, leaf: int = 32, tol: float = 1e-12,
                   lo: float = 0.0, hi: float = 1.0) -> GPProblem:
    """Generic seeded problem: points ~ U([lo,hi]^dim) (1-D sorted), y ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    if dim == 1:
        x = np.sort(rng.uniform(lo, hi, size=n)).reshape(n, 1)
    else:
        x = rng.uniform(lo, hi, size=(n, dim))
    y = rng.standard_normal(n)
    return GPProblem("rand_d%d_k%d_n%d_s%d" % (dim, kernel, n, seed), x.astype(np.float64),
                     y, kernel, (a, ell), sigma2, leaf, tol)


def regression_model(n: int = 1024, tol: float = 1e-8, leaf: int = 20,
                     seed: int = 56) -> GPProblem:
    """The regression experiment of §5.6: x ~ U(-3, 3) sorted, y = sin(2x) +
    exp(x) / 8 plus N(0, 1) noise, kernel exp(-(x - x')^2) (SE with a = 1,
    l = 1/sqrt(2)), noise variance 1, smallest blocks of 20 points; the
    factorization precision is the parameter the experiment varies.  The
    paper's own draw is not published, so this is a fresh seeded draw."""
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(-3.0, 3.0, n))
    y = np.sin(2.0 * x) + np.exp(x) / 8.0 + rng.standard_normal(n)
    return GPProblem("regression_n%d_tol%g_leaf%d" % (n, tol, leaf), x.reshape(n, 1), y, K_SE,
                     (1.0, 1.0 / math.sqrt(2.0)), 1.0, leaf, tol)


def paper_table(kind: int, n: int, dim: int = 1, seed: int = 101) -> GPProblem:
    """The test problems of §5's timing tables: r ~ U([-3, 3]^dim) and
    C_ij = s delta_ij + k(r_i, r_j) with the table's kernel:
    Gaussian exp(-|r|^2) (SE, a = 1, l = 1/sqrt(2)) with s = 2; exponential
    exp(-|r|) (a = 1, l = 1) with s = 1; inverse multiquadric
    1/sqrt(1 + |r|^2) (a = 1, l = 1) with s = 1.  ``y`` holds the known
    solution x of the test problem C x = b (N(0, 1) entries); b is formed from
    it by the caller.  Smallest blocks of 64 points, tolerance 1e-14."""
    params = {K_SE: ((1.0, 1.0 / math.sqrt(2.0)), 2.0), K_EXP: ((1.0, 1.0), 1.0),
              K_IMQ: ((1.0, 1.0), 1.0)}
    theta, s = params[kind]
    rng = np.random.default_rng(seed)
    x = rng.uniform(-3.0, 3.0, size=(n, dim))
    if dim == 1:
        x = np.sort(x, axis=0)
    xt = rng.standard_normal(n)
    return GPProblem("table_k%d_d%d_n%d" % (kind, dim, n), x.astype(np.float64), xt, kind,
                     theta, s, 64, 1e-14)
