"""Pins for the numpy walk-through of the HODLR method (oracle/hodlr_ref.py).

These check the method's intermediate quantities against what the
mathematics fixes: the factor list multiplies back to C (§3.2), each
coupling determinant equals a ratio of dense determinants (Sylvester's
theorem, §4), leaf size does not change the result (§5.6), exact-rank
kernels give exact answers, and cross approximation meets its tolerance.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import hodlr_ref as hr
import workloads as wl


def _ld(C):
    s, v = np.linalg.slogdet(C)
    assert s > 0
    return v


def test_levels_and_tree():
    assert hr.num_levels(2048, 64) == 5
    assert hr.num_levels(1 << 20, 128) == 13
    assert hr.num_levels(1 << 22, 256) == 14
    assert hr.num_levels(100, 100) == 0
    assert hr.num_levels(101, 100) == 1
    nodes = hr.tree_nodes(1000, hr.num_levels(1000, 64))
    for level in nodes:
        assert level[0][0] == 0 and level[-1][1] == 1000
        assert all(level[i][1] == level[i + 1][0] for i in range(len(level) - 1))
    assert max(e - s for s, e in nodes[-1]) <= 64


def test_kd_order_is_a_median_split():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (777, 2))
    leaf = 20
    perm = hr.kd_order(x, leaf)
    assert np.array_equal(np.sort(perm), np.arange(777))
    xs = x[perm]
    nodes = hr.tree_nodes(777, hr.num_levels(777, leaf))
    for d, level in enumerate(nodes[:-1]):
        c = d % 2
        for (s, e) in level:
            m = s + (e - s) // 2
            if m > s and e > m:
                assert xs[s:m, c].max() <= xs[m:e, c].min()


def test_aca_exact_rank_blocks():
    rng = np.random.default_rng(2)
    xa = np.sort(rng.uniform(0, 1, 60)).reshape(-1, 1)
    xb = np.sort(rng.uniform(1, 2, 50)).reshape(-1, 1)
    for kind, rmax in [(wl.K_CONST, 1), (wl.K_EXP, 1), (wl.K_MATERN32, 2)]:
        A = hr.kernel_block(kind, xa, xb, 1.0, 0.5)
        U, V, cap = hr.aca(lambda i: A[i], lambda j: A[:, j], 60, 50, 1e-13, 30)
        # the exact-rank terms plus at most one term below tolerance
        assert U.shape[1] <= rmax + 1 and not cap
        assert np.linalg.norm(A - U @ V.T) <= 1e-13 * np.linalg.norm(A)


@pytest.mark.parametrize("tol", [1e-4, 1e-8, 1e-12])
def test_aca_meets_tolerance_on_smooth_block(tol):
    rng = np.random.default_rng(3)
    xa = rng.uniform(0, 1, (120, 2))
    xb = rng.uniform(1.2, 2, (90, 2))
    A = hr.kernel_block(wl.K_SE, xa, xb, 1.0, 0.5)
    U, V, _ = hr.aca(lambda i: A[i], lambda j: A[:, j], 120, 90, tol, 90)
    err = np.linalg.norm(A - U @ V.T) / np.linalg.norm(A)
    assert err <= 10 * tol
    sv = np.linalg.svd(A, compute_uv=False)
    # ACA's rank is close to the optimal (SVD) rank at this accuracy
    assert U.shape[1] <= int(np.sum(sv > 0.1 * tol * sv[0])) + 3


def test_single_level_is_dense_cholesky():
    p = wl.se1d_small(256)
    ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=256, tol=1e-12, presorted=True)
    assert ref.L == 0
    d = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    out = ref.loglik(p.y)
    assert out["logdet"] == pytest.approx(d["logdet"], rel=1e-14)
    assert np.linalg.norm(out["alpha"] - d["alpha"]) <= 1e-12 * np.linalg.norm(d["alpha"])


@pytest.mark.parametrize("L", [1, 2, 3])
def test_factor_list_multiplies_back_to_C(L):
    """K_L B_{L-1} ... B_0 reproduces C to cross-approximation accuracy."""
    n = 96
    p = wl.random_problem(n, 1, wl.K_SE, seed=11, ell=0.3, sigma2=0.05, lo=-1, hi=1)
    ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=n >> L, tol=1e-14, presorted=True)
    assert ref.L == L
    prod = np.eye(n)
    for F in ref.factor_matrices():
        prod = prod @ F
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    assert np.linalg.norm(prod - C) <= 1e-12 * np.linalg.norm(C)
    # each factor B_d is block diagonal with 2^d identity-plus-low-rank blocks
    for d, B in zip(range(L - 1, -1, -1), ref.factor_matrices()[1:]):
        for i, (s, e) in enumerate(ref.nodes[d]):
            off = B[s:e].copy()
            off[:, s:e] = 0
            assert np.all(off == 0)
            r = ref.ranks[d][i]
            assert np.linalg.matrix_rank(B[s:e, s:e] - np.eye(e - s), tol=1e-10) <= 2 * r


def test_one_level_formula():
    """L = 1: log det C = log det A11 + log det A22 + log det(I - Q P) with
    P = V^T A22^{-1} V, Q = U^T A11^{-1} U (Sylvester on the one-level
    factorization of §3.2)."""
    n = 80
    p = wl.random_problem(n, 1, wl.K_MATERN32, seed=12, ell=0.4, sigma2=0.1)
    ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=40, tol=1e-14, presorted=True)
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    U, V = ref.W[1][0], ref.W[1][1]
    A11, A22 = C[:40, :40], C[40:, 40:]
    P = V.T @ np.linalg.solve(A22, V)
    Q = U.T @ np.linalg.solve(A11, U)
    expect = _ld(A11) + _ld(A22) + _ld(np.eye(P.shape[0]) - Q @ P)
    assert ref.logdet() == pytest.approx(expect, rel=1e-13)
    assert ref.logdet() == pytest.approx(_ld(C), rel=1e-13)


def test_per_node_sylvester_identity():
    """log det M_tau = log det C_tau - log det C_alpha - log det C_beta <= 0."""
    p = wl.random_problem(300, 2, wl.K_SE, seed=13, ell=0.25, sigma2=0.05)
    ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=40, tol=1e-14, max_rank=150)
    assert ref.capped == 0
    C = oracle.dense_matrix(ref.xs, p.kernel, p.theta, p.sigma2)
    for d in range(ref.L):
        for i, (s, e) in enumerate(ref.nodes[d]):
            m = s + (e - s) // 2
            expect = _ld(C[s:e, s:e]) - _ld(C[s:m, s:m]) - _ld(C[m:e, m:e])
            got = ref.node_logdet[d][i]
            assert got == pytest.approx(expect, rel=1e-9, abs=1e-10)
            assert got <= 1e-12


def test_leaf_size_does_not_change_result():
    p = wl.se1d_small(1024)
    lds = []
    for leaf in (16, 32, 64, 128, 256):
        ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=leaf, tol=1e-13, presorted=True)
        lds.append(ref.logdet())
    assert max(lds) - min(lds) <= 1e-11 * abs(lds[0])


def test_exact_rank_matern_gives_exact_result():
    p = wl.matern1d(4096)
    ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=128, tol=1e-10, presorted=True)
    assert max(max(r) for r in ref.ranks) <= 3
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2)
    out = ref.loglik(p.y)
    assert abs(out["logdet"] - kf["logdet"]) <= 1e-13 * abs(kf["logdet"])
    assert np.linalg.norm(out["alpha"] - kf["alpha"]) <= 1e-10 * np.linalg.norm(kf["alpha"])


def test_error_shrinks_with_tolerance():
    p = wl.se1d_small(1024)
    d = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    errs = []
    for tol in (1e-4, 1e-7, 1e-10):
        ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=64, tol=tol, presorted=True)
        errs.append(abs(ref.logdet() - d["logdet"]) / abs(d["logdet"]))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] <= 1e-9


def test_small_config_meets_fp64_bars():
    """n = 2048 SE workload: relative log-det error <= 1e-10 and relative
    residual ||y - C x|| / ||y|| <= 1e-10 against the dense oracle."""
    p = wl.se1d_small()
    ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=p.leaf, tol=p.tol, presorted=True)
    d = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    out = ref.loglik(p.y)
    assert abs(out["logdet"] - d["logdet"]) <= 1e-10 * abs(d["logdet"])
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    assert np.linalg.norm(p.y - C @ out["alpha"]) <= 1e-10 * np.linalg.norm(p.y)


def test_solve_in_caller_order_for_2d():
    p = wl.random_problem(500, 2, wl.K_MATERN32, seed=14, ell=0.2, sigma2=0.1)
    ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=32, tol=1e-12, max_rank=300)
    assert ref.capped == 0
    d = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    out = ref.loglik(p.y)
    assert out["logdet"] == pytest.approx(d["logdet"], rel=1e-10)
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    assert np.linalg.norm(p.y - C @ out["alpha"]) <= 1e-10 * np.linalg.norm(p.y)


def test_rank_cap_is_reported_and_costs_accuracy():
    p = wl.random_problem(500, 2, wl.K_MATERN32, seed=14, ell=0.2, sigma2=0.1)
    ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf=32, tol=1e-12, max_rank=64)
    assert ref.capped > 0
    assert max(max(r) for r in ref.ranks) == 64
