"""Pins for the dense FP64 oracle and the Kalman oracle.

Each check compares the oracle with something the mathematics fixes on its
own: closed forms, brute-force determinants, determinant bounds, scaling
laws, or an independent library routine (LAPACK through numpy).  A plausible
mistake in the oracle (a dropped noise term, a wrong kernel constant, a
missing factor 2 in the log-det, a transposed triangular solve, a wrong
state-space transition) fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import hodlr_ref
import workloads as wl

KINDS = [wl.K_SE, wl.K_MATERN32, wl.K_EXP, wl.K_CONST, wl.K_IMQ]


def test_kernel_closed_forms(oracle_lib):
    a, ell = 1.7, 0.4
    e = math.e
    # SE at r = l is a^2 e^{-1/2}; Matern-3/2 at r = l/sqrt(3) is 2 a^2 / e;
    # exponential at r = l is a^2 / e; constant is a^2 everywhere.
    assert oracle.kernel_value(wl.K_SE, [0.0], [ell], a, ell) == pytest.approx(a * a / math.sqrt(e), rel=1e-15)
    assert oracle.kernel_value(wl.K_MATERN32, [0.2], [0.2 + ell / math.sqrt(3)], a, ell) == \
        pytest.approx(2 * a * a / e, rel=1e-14)
    assert oracle.kernel_value(wl.K_EXP, [1.0], [1.0 - ell], a, ell) == pytest.approx(a * a / e, rel=1e-14)
    assert oracle.kernel_value(wl.K_CONST, [3.0], [-9.0], a, ell) == a * a
    # inverse multiquadric: 1 / sqrt(1 + 3) = 1/2 at r = sqrt(3) l, 1/3 at
    # r = sqrt(8) l (in 2-D: the offset (2 l, 2 l))
    assert oracle.kernel_value(wl.K_IMQ, [0.5], [0.5 + math.sqrt(3) * ell], a, ell) == \
        pytest.approx(a * a / 2, rel=1e-15)
    assert oracle.kernel_value(wl.K_IMQ, [0.0, 0.0], [2 * ell, 2 * ell], a, ell) == \
        pytest.approx(a * a / 3, rel=1e-15)
    # Euclidean distance in 2-D and 3-D: |(3,4)| = 5, |(1,2,2)| = 3
    assert oracle.kernel_value(wl.K_EXP, [0.0, 0.0], [3.0, 4.0], 1.0, 5.0) == pytest.approx(1 / e, rel=1e-15)
    assert oracle.kernel_value(wl.K_EXP, [0, 0, 0], [1, 2, 2], 1.0, 3.0) == pytest.approx(1 / e, rel=1e-15)
    for k in KINDS:
        assert oracle.kernel_value(k, [0.3, 0.1], [0.3, 0.1], a, ell) == pytest.approx(a * a, rel=1e-15)


def test_inverse_multiquadric_is_a_gaussian_scale_mixture(oracle_lib):
    # (1 + u)^(-1/2) = pi^(-1/2) int_0^inf t^(-1/2) exp(-t (1 + u)) dt, evaluated
    # by quadrature (substitution t = s^2 removes the endpoint singularity)
    from scipy.integrate import quad
    a, ell = 0.8, 0.3
    for r in (0.0, 0.1, 0.45, 2.0, 17.0):
        u = (r / ell) ** 2
        val, _ = quad(lambda s_: 2.0 * math.exp(-s_ * s_ * (1.0 + u)), 0.0, math.inf,
                      epsabs=0.0, epsrel=1e-13)
        assert oracle.kernel_value(wl.K_IMQ, [1.0], [1.0 + r], a, ell) == \
            pytest.approx(a * a * val / math.sqrt(math.pi), rel=1e-12)


def test_numpy_kernel_agrees_with_c_kernel(oracle_lib):
    rng = np.random.default_rng(0)
    for dim in (1, 2, 3):
        xa = rng.uniform(-1, 1, (7, dim))
        xb = rng.uniform(-1, 1, (5, dim))
        for k in KINDS:
            blk = hodlr_ref.kernel_block(k, xa, xb, 1.3, 0.35)
            for i in range(7):
                for j in range(5):
                    assert blk[i, j] == pytest.approx(oracle.kernel_value(k, xa[i], xb[j], 1.3, 0.35),
                                                      rel=1e-14, abs=1e-300)


def test_dense_matrix_symmetric_with_noise_on_diagonal(oracle_lib):
    p = wl.random_problem(50, 2, wl.K_MATERN32, seed=3)
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    assert np.array_equal(C, C.T)
    assert np.allclose(np.diag(C), p.theta[0] ** 2 + p.sigma2, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [1, 5, 64, 300])
def test_zero_kernel_is_scaled_identity(oracle_lib, n):
    p = wl.random_problem(n, 1, wl.K_SE, seed=n)
    s2 = 0.37
    out = oracle.gp_dense(p.x, p.y, wl.K_SE, (0.0, 0.2), s2)
    assert out["logdet"] == pytest.approx(n * math.log(s2), rel=1e-14)
    assert np.allclose(out["alpha"], p.y / s2, rtol=1e-14, atol=0)
    quad = float(p.y @ p.y) / s2
    assert out["quad"] == pytest.approx(quad, rel=1e-13)
    assert out["loglik"] == pytest.approx(-0.5 * quad - 0.5 * n * math.log(s2) - 0.5 * n * math.log(2 * math.pi),
                                          rel=1e-13)


@pytest.mark.parametrize("n", [1, 17, 256, 1000])
def test_rank_one_kernel_determinant_lemma_and_sherman_morrison(oracle_lib, n):
    p = wl.rank1_points(n)
    a, s2 = p.theta[0], p.sigma2
    out = oracle.gp_dense(p.x, p.y, wl.K_CONST, p.theta, s2)
    # C = s2 I + a^2 1 1^T: det C = s2^n (1 + n a^2 / s2)
    assert out["logdet"] == pytest.approx(n * math.log(s2) + math.log1p(n * a * a / s2), rel=1e-13)
    # C^{-1} y = (y - a^2 (1^T y) / (s2 + n a^2) 1) / s2
    alpha = (p.y - a * a * p.y.sum() / (s2 + n * a * a)) / s2
    assert np.allclose(out["alpha"], alpha, rtol=1e-11, atol=1e-12)


def _leibniz_det(A):
    n = A.shape[0]
    total = 0.0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        prod = 1.0
        for i in range(n):
            prod *= A[i, perm[i]]
        total += (-1) ** inv * prod
    return total


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_brute_force_determinant(oracle_lib, kind, n):
    p = wl.random_problem(n, 2, kind, seed=10 + n, ell=0.5, sigma2=0.2)
    C = oracle.dense_matrix(p.x, kind, p.theta, p.sigma2)
    det = _leibniz_det(C)
    out = oracle.gp_dense(p.x, p.y, kind, p.theta, p.sigma2)
    assert out["logdet"] == pytest.approx(math.log(det), rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("kind", KINDS)
def test_determinant_bounds(oracle_lib, kind):
    p = wl.random_problem(200, 1, kind, seed=5, a=1.2, ell=0.05, sigma2=0.3)
    out = oracle.gp_dense(p.x, p.y, kind, p.theta, p.sigma2)
    # every eigenvalue >= sigma^2 (K is PSD); Hadamard: det <= prod of diagonal
    assert out["logdet"] >= 200 * math.log(0.3) - 1e-9
    assert out["logdet"] <= 200 * math.log(1.2 ** 2 + 0.3) + 1e-9


def test_homogeneity(oracle_lib):
    p = wl.random_problem(150, 2, wl.K_MATERN32, seed=8, a=0.9, ell=0.2, sigma2=0.05)
    c = 3.0
    o1 = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    o2 = oracle.gp_dense(p.x, p.y, p.kernel, (c * p.theta[0], p.theta[1]), c * c * p.sigma2)
    assert o2["logdet"] == pytest.approx(o1["logdet"] + 2 * 150 * math.log(c), rel=1e-13)
    assert np.allclose(o2["alpha"], o1["alpha"] / c ** 2, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("kind", KINDS)
def test_lapack_cross_check(oracle_lib, dim, kind):
    p = wl.random_problem(400, dim, kind, seed=20 + dim, ell=0.3, sigma2=0.02)
    out = oracle.gp_dense(p.x, p.y, kind, p.theta, p.sigma2)
    C = oracle.dense_matrix(p.x, kind, p.theta, p.sigma2)
    sign, ld = np.linalg.slogdet(C)
    assert sign > 0
    assert out["logdet"] == pytest.approx(ld, rel=1e-12, abs=1e-10)
    alpha = np.linalg.solve(C, p.y)
    assert np.linalg.norm(out["alpha"] - alpha) <= 1e-9 * np.linalg.norm(alpha)
    G = oracle.cholesky(C)
    assert np.allclose(G @ G.T, C, rtol=0, atol=1e-13)
    assert np.array_equal(np.triu(G, 1), np.zeros_like(G))


def test_cholesky_rejects_indefinite(oracle_lib):
    with pytest.raises(oracle.OracleError):
        oracle.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    # a covariance with negative noise large enough to lose definiteness
    p = wl.random_problem(20, 1, wl.K_SE, seed=1)
    with pytest.raises(oracle.OracleError):
        oracle.gp_dense(p.x, p.y, wl.K_SE, (1.0, 0.3), -2.0)


def test_matvec_rows_matches_dense_product(oracle_lib):
    p = wl.random_problem(300, 2, wl.K_SE, seed=9, ell=0.2, sigma2=0.1)
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    v = np.random.default_rng(1).standard_normal(300)
    rows = np.array([0, 5, 17, 299, 150])
    got = oracle.matvec_rows(p.x, p.kernel, p.theta, p.sigma2, v, rows)
    assert np.allclose(got, (C @ v)[rows], rtol=1e-13, atol=1e-13)


def test_kalman_one_and_two_points(oracle_lib):
    a, ell, s2 = 1.3, 0.7, 0.2
    y1 = np.array([0.9])
    o = oracle.kalman_matern32([0.4], y1, (a, ell), s2)
    assert o["logdet"] == pytest.approx(math.log(a * a + s2), rel=1e-15)
    assert o["quad"] == pytest.approx(0.81 / (a * a + s2), rel=1e-15)
    assert o["alpha"][0] == pytest.approx(0.9 / (a * a + s2), rel=1e-14)
    # two points: explicit 2x2 determinant and inverse
    t = np.array([0.1, 0.5])
    y = np.array([0.3, -1.1])
    s = math.sqrt(3) * 0.4 / ell
    k = a * a * (1 + s) * math.exp(-s)
    d = a * a + s2
    det = d * d - k * k
    o = oracle.kalman_matern32(t, y, (a, ell), s2)
    assert o["logdet"] == pytest.approx(math.log(det), rel=1e-14)
    alpha = np.array([d * y[0] - k * y[1], -k * y[0] + d * y[1]]) / det
    assert np.allclose(o["alpha"], alpha, rtol=1e-13)
    assert o["quad"] == pytest.approx(float(y @ alpha), rel=1e-13)


@pytest.mark.parametrize("n", [64, 1000, 4096])
def test_kalman_matches_dense(oracle_lib, n):
    p = wl.matern1d(n)
    dn = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2)
    assert kf["logdet"] == pytest.approx(dn["logdet"], rel=1e-12)
    assert kf["quad"] == pytest.approx(dn["quad"], rel=1e-12)
    assert np.linalg.norm(kf["alpha"] - dn["alpha"]) <= 1e-10 * np.linalg.norm(dn["alpha"])
    assert kf["loglik"] == pytest.approx(dn["loglik"], rel=1e-12)


def test_kalman_rejects_unsorted(oracle_lib):
    with pytest.raises(oracle.OracleError):
        oracle.kalman_matern32([0.0, 1.0, 0.5], [1.0, 2.0, 3.0], (1.0, 1.0), 0.1)


def _golden_rows(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = []
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            n, err = line.split()
            rows.append((int(n), float(err)))
    return rows


TABLES = [("gaussian_1d_solution_error.txt", wl.K_SE),
          ("exponential_1d_solution_error.txt", wl.K_EXP),
          ("imq_1d_solution_error.txt", wl.K_IMQ)]


@pytest.mark.parametrize("kind,n,err", [(k, n, e) for f, k in TABLES for n, e in _golden_rows(f)
                                        if n <= 20000])
def test_walkthrough_meets_the_papers_tables(oracle_lib, kind, n, err):
    # §5's timing tables (one-dimensional Gaussian, exponential and inverse
    # multiquadric): the solution error of the method's own steps
    # (walk-through) on the table's test problem, with b formed from the known
    # x by the oracle's exact product, is within a factor 10 of the printed
    # value (the tables give orders of magnitude)
    p = wl.paper_table(kind, n)
    b = oracle.matvec_rows(p.x, p.kernel, p.theta, p.sigma2, p.y, np.arange(n))
    ref = hodlr_ref.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, p.leaf, p.tol)
    xs = ref.solve(b)
    rel = np.linalg.norm(xs - p.y) / np.linalg.norm(p.y)
    assert rel <= 10 * err, rel
