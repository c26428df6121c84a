"""Pins of the oracle's per-point noise (§5: the diagonal of C is
sigma_i^2, C_ij = sigma_i^2 delta_ij + k(x_i, x_j); here sigma^2 + sigma_i^2)
to what the mathematics fixes, independent of the oracle's own code path:

* K = 0: C is the diagonal itself;
* constant kernel: matrix determinant lemma and Sherman-Morrison with a
  diagonal D in place of sigma^2 I;
* a uniform per-point variance c equals the scalar noise sigma^2 + c;
* Leibniz determinants for n <= 5;
* the dense definition and the state-space (Kalman) recursion, two unrelated
  algorithms, agree for Matern-3/2 with heteroscedastic noise.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def _noise(n, seed):
    return np.random.default_rng(seed).uniform(0.01, 2.0, n)


def test_zero_kernel_gives_the_diagonal(oracle_lib):
    p = wl.random_problem(40, 1, wl.K_SE, seed=1)
    d = 0.2 + _noise(40, 2)
    out = oracle.gp_dense_noise(p.x, p.y, wl.K_SE, (0.0, 0.3), 0.2, d - 0.2)
    assert out["logdet"] == pytest.approx(float(np.sum(np.log(d))), rel=1e-14)
    assert np.allclose(out["alpha"], p.y / d, rtol=1e-14, atol=0)


@pytest.mark.parametrize("n", [1, 9, 300])
def test_constant_kernel_closed_forms(oracle_lib, n):
    # C = D + a^2 1 1^T: det C = det D (1 + a^2 sum 1/d_i),
    # C^{-1} y = D^{-1} y - a^2 D^{-1} 1 (1^T D^{-1} y) / (1 + a^2 sum 1/d_i)
    p = wl.rank1_points(n)
    a, s2 = p.theta[0], p.sigma2
    nz = _noise(n, 3)
    d = s2 + nz
    out = oracle.gp_dense_noise(p.x, p.y, wl.K_CONST, p.theta, s2, nz)
    g = 1.0 + a * a * float(np.sum(1.0 / d))
    assert out["logdet"] == pytest.approx(float(np.sum(np.log(d))) + math.log(g), rel=1e-13)
    w = p.y / d
    alpha = w - a * a * (1.0 / d) * float(np.sum(w)) / g
    assert np.allclose(out["alpha"], alpha, rtol=1e-11, atol=1e-13)
    assert out["quad"] == pytest.approx(float(p.y @ w) - a * a * float(np.sum(w)) ** 2 / g, rel=1e-11)


def test_uniform_per_point_variance_is_scalar_noise(oracle_lib):
    p = wl.random_problem(200, 2, wl.K_MATERN32, seed=4, ell=0.3, sigma2=0.05)
    c = 0.125
    o1 = oracle.gp_dense_noise(p.x, p.y, p.kernel, p.theta, p.sigma2, np.full(p.n, c))
    o2 = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2 + c)
    assert o1["logdet"] == pytest.approx(o2["logdet"], rel=1e-13)
    assert np.allclose(o1["alpha"], o2["alpha"], rtol=1e-11, atol=1e-13)
    t = p.x[:, 0].copy()
    t.sort()
    k1 = oracle.kalman_matern32(t, p.y, p.theta, p.sigma2, noise=np.full(p.n, c))
    k2 = oracle.kalman_matern32(t, p.y, p.theta, p.sigma2 + c)
    assert k1["logdet"] == pytest.approx(k2["logdet"], rel=1e-14)
    assert np.allclose(k1["alpha"], k2["alpha"], rtol=1e-13, atol=1e-15)


def _leibniz_det(C):
    n = C.shape[0]
    tot = 0.0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        term = -1.0 if inv % 2 else 1.0
        for i in range(n):
            term *= C[i, perm[i]]
        tot += term
    return tot


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_brute_force_determinant(oracle_lib, n):
    p = wl.random_problem(n, 2, wl.K_SE, seed=30 + n, ell=0.5, sigma2=0.1)
    nz = _noise(n, 5)
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2) + np.diag(nz)
    out = oracle.gp_dense_noise(p.x, p.y, p.kernel, p.theta, p.sigma2, nz)
    assert out["logdet"] == pytest.approx(math.log(_leibniz_det(C)), rel=1e-12, abs=1e-12)


def test_kalman_and_dense_agree_with_heteroscedastic_noise(oracle_lib):
    p = wl.matern1d(400)
    nz = _noise(p.n, 6)
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, noise=nz)
    dn = oracle.gp_dense_noise(p.x, p.y, p.kernel, p.theta, p.sigma2, nz)
    assert kf["logdet"] == pytest.approx(dn["logdet"], rel=1e-12)
    assert kf["quad"] == pytest.approx(dn["quad"], rel=1e-11)
    assert np.allclose(kf["alpha"], dn["alpha"], rtol=1e-9, atol=1e-11)
