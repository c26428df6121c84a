"""Pins for the dense gradient oracle (oracle/grad_ref.py).

* The a and sigma^2 components against a closed form in the eigenvalues of the
  unit-amplitude kernel matrix K1 (C = a^2 K1 + sigma^2 I = V diag(mu) V^T with
  mu_i = a^2 lambda_i + sigma^2, c = V^T y):
      L = -1/2 sum log mu_i - 1/2 sum c_i^2 / mu_i - n/2 log 2 pi,
      dL/dp = sum (c_i^2 / mu_i^2 - 1 / mu_i) / 2 * dmu_i/dp,
  dmu_i/da = 2 a lambda_i, dmu_i/dsigma2 = 1 (numpy's symmetric eigensolver,
  no Cholesky and no trace).
* The l component against a fourth-order central difference of the dense
  likelihood (oracle.gp_dense, the plain Cholesky definition), for every kernel.
A dropped factor (the 1/2, the 2 of d(a^2)/da), a wrong sign of the trace term
or a wrong kernel derivative fails one of them.
"""
import numpy as np
import pytest

import oracle
from oracle import grad_ref
import workloads as wl

KINDS = [wl.K_SE, wl.K_MATERN32, wl.K_EXP, wl.K_IMQ]


def _problem(n, dim, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, (n, dim))
    y = rng.standard_normal(n)
    return x, y


@pytest.mark.parametrize("kind", KINDS + [wl.K_CONST])
def test_amplitude_and_noise_components_match_eigen_closed_form(oracle_lib, kind):
    x, y = _problem(150, 2, 11 + kind)
    a, ell, s2 = 1.3, 0.2, 0.05
    K1 = oracle.dense_matrix(x, kind, (1.0, ell), 0.0)
    lam, V = np.linalg.eigh(K1)
    c = V.T @ y
    mu = a * a * lam + s2
    w = 0.5 * (c * c / (mu * mu) - 1.0 / mu)
    ga = np.sum(w * 2.0 * a * lam)
    gs = np.sum(w)
    L = -0.5 * np.sum(np.log(mu)) - 0.5 * np.sum(c * c / mu) - 0.5 * len(y) * np.log(2 * np.pi)
    g = grad_ref.gp_dense_grad(x, y, kind, (a, ell), s2)
    assert g["loglik"] == pytest.approx(L, rel=1e-11)
    assert g["grad"][0] == pytest.approx(ga, rel=1e-9, abs=1e-9)
    assert g["grad"][2] == pytest.approx(gs, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("dim", [1, 2])
def test_length_scale_component_matches_fourth_order_difference(oracle_lib, kind, dim):
    x, y = _problem(120, dim, 40 + 3 * kind + dim)
    a, ell, s2 = 0.9, 0.15, 0.02
    h = 1e-3 * ell

    def L(e):
        return oracle.gp_dense(x, y, kind, (a, e), s2)["loglik"]

    fd = (-L(ell + 2 * h) + 8 * L(ell + h) - 8 * L(ell - h) + L(ell - 2 * h)) / (12 * h)
    g = grad_ref.gp_dense_grad(x, y, kind, (a, ell), s2)["grad"][1]
    assert g == pytest.approx(fd, rel=1e-7, abs=1e-6)


def test_constant_kernel_has_no_length_scale_dependence(oracle_lib):
    x, y = _problem(60, 1, 5)
    g = grad_ref.gp_dense_grad(x, y, wl.K_CONST, (1.1, 0.3), 0.1)["grad"]
    assert g[1] == 0.0
