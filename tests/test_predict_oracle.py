"""Pins of the oracle's prediction (§2.1, predictive mean and variance) to
what the mathematics fixes, independent of its own code path:

* constant (rank-one) kernel: closed forms through Sherman-Morrison;
* one training point: scalar closed forms;
* points so far apart that every cross-covariance underflows to zero in FP64
  (K = a^2 I exactly): closed forms at a training point and far away;
* invariance under reordering the training data;
* interpolation: with sigma^2 -> 0 the mean reproduces the data and the
  variance vanishes at the training points.
"""
import numpy as np
import pytest

import oracle
import workloads as wl


def test_constant_kernel_closed_form():
    # K = a^2 1 1^T: C^{-1} = (I - a^2 1 1^T / (s2 + n a^2)) / s2, so at any input
    # mean = a^2 sum(y) / (s2 + n a^2) and var = a^2 s2 / (s2 + n a^2)
    rng = np.random.default_rng(5)
    n, a, s2 = 40, 0.7, 0.3
    x = np.sort(rng.uniform(0, 1, n)).reshape(-1, 1)
    y = rng.standard_normal(n)
    xt = np.array([[-3.0], [0.4], [17.0]])
    mean, var = oracle.gp_predict_dense(x, y, xt, wl.K_CONST, (a, 1.0), s2)
    a2 = a * a
    assert mean == pytest.approx(np.full(3, a2 * y.sum() / (s2 + n * a2)), rel=1e-13)
    assert var == pytest.approx(np.full(3, a2 * s2 / (s2 + n * a2)), rel=1e-12)


@pytest.mark.parametrize("kind", [wl.K_SE, wl.K_MATERN32, wl.K_EXP])
def test_one_training_point_closed_form(kind):
    a, ell, s2 = 1.3, 0.8, 0.2
    x = np.array([[0.25]])
    y = np.array([1.7])
    xt = np.array([[0.25], [0.9], [3.0]])
    mean, var = oracle.gp_predict_dense(x, y, xt, kind, (a, ell), s2)
    d = np.abs(xt[:, 0] - 0.25)
    if kind == wl.K_SE:
        k = a * a * np.exp(-d * d / (2 * ell * ell))
    elif kind == wl.K_MATERN32:
        s = np.sqrt(3.0) * d / ell
        k = a * a * (1 + s) * np.exp(-s)
    else:
        k = a * a * np.exp(-d / ell)
    den = a * a + s2
    assert mean == pytest.approx(k * y[0] / den, rel=1e-13, abs=1e-300)
    assert var == pytest.approx(a * a - k * k / den, rel=1e-13)


def test_separated_points_closed_form():
    # SE with l = 0.01 and spacing 10: exp(-10^2 / (2e-4)) underflows to 0, so
    # K = a^2 I exactly and every point is predicted from itself alone
    a, s2 = 1.1, 0.05
    x = (10.0 * np.arange(6)).reshape(-1, 1)
    y = np.array([0.3, -1.0, 2.0, 0.5, -0.7, 1.2])
    xt = np.vstack([x, [[1e3]]])
    mean, var = oracle.gp_predict_dense(x, y, xt, wl.K_SE, (a, 0.01), s2)
    a2 = a * a
    assert mean[:6] == pytest.approx(a2 * y / (a2 + s2), rel=1e-14)
    assert var[:6] == pytest.approx(np.full(6, a2 * s2 / (a2 + s2)), rel=1e-13)
    assert mean[6] == 0.0 and var[6] == pytest.approx(a2, rel=1e-15)


def test_reordering_the_data_changes_nothing():
    p = wl.random_problem(300, 2, wl.K_MATERN32, seed=11, ell=0.3, sigma2=0.05)
    xt = np.random.default_rng(12).uniform(-0.2, 1.2, (20, 2))
    m1, v1 = oracle.gp_predict_dense(p.x, p.y, xt, p.kernel, p.theta, p.sigma2)
    perm = np.random.default_rng(13).permutation(p.n)
    m2, v2 = oracle.gp_predict_dense(p.x[perm], p.y[perm], xt, p.kernel, p.theta, p.sigma2)
    assert np.max(np.abs(m1 - m2)) <= 1e-11 * np.max(np.abs(m1))
    assert np.max(np.abs(v1 - v2)) <= 1e-11


def test_interpolation_limit():
    # noise -> 0: the posterior mean passes through the data and the variance
    # of f vanishes there (Matern-3/2, points about one length scale apart)
    rng = np.random.default_rng(21)
    n = 25
    x = np.sort(rng.uniform(0, 25, n)).reshape(-1, 1)
    y = rng.standard_normal(n)
    mean, var = oracle.gp_predict_dense(x, y, x, wl.K_MATERN32, (1.0, 1.0), 1e-12)
    assert np.max(np.abs(mean - y)) <= 1e-8
    assert np.max(np.abs(var)) <= 1e-8


def test_regression_estimate_at_the_data():
    # at the training points K C^{-1} = I - sigma^2 C^{-1}, so the regression
    # estimate of §5.6 equals y - sigma^2 C^{-1} y (C^{-1} y by LAPACK here,
    # independent of the oracle's Cholesky)
    p = wl.regression_model(256)
    yhat, _ = oracle.gp_predict_dense(p.x, p.y, p.x, p.kernel, p.theta, p.sigma2, want_var=False)
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    alpha = np.linalg.solve(C, p.y)
    assert np.max(np.abs(yhat - (p.y - p.sigma2 * alpha))) <= 1e-12 * np.max(np.abs(p.y))


def test_walkthrough_rmse_difference_follows_tolerance():
    # §5.6: the RMSE of the regression through the HODLR factor differs from the
    # exact one by an amount proportional to the factorization precision, for
    # any size of the smallest blocks (walk-through of the method against the
    # dense oracle)
    from oracle import hodlr_ref as hr
    p = wl.regression_model()
    n = p.n
    exact, _ = oracle.gp_predict_dense(p.x, p.y, p.x, p.kernel, p.theta, p.sigma2, want_var=False)
    rm_exact = np.linalg.norm(p.y - exact) / np.sqrt(n)
    Ks = oracle.cross_matrix(p.x, p.x, p.kernel, p.theta)
    errs = {}
    for tol in (1e-4, 1e-7, 1e-10):
        for leaf in (20, 64):
            ref = hr.HodlrRef(p.x, p.kernel, p.theta, p.sigma2, leaf, tol)
            yh = Ks @ ref.solve(p.y)
            d = abs(np.linalg.norm(p.y - yh) / np.sqrt(n) - rm_exact)
            e = np.max(np.abs(yh - exact))
            assert d <= 1e-2 * tol + 1e-14, (tol, leaf, d)
            assert e <= 10 * tol, (tol, leaf, e)
            errs[tol, leaf] = e
    for leaf in (20, 64):
        assert errs[1e-4, leaf] > errs[1e-7, leaf] > errs[1e-10, leaf]
