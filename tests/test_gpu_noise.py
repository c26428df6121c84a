"""GPU parity with per-point noise variances (§5: the diagonal of C is
sigma_i^2; here sigma^2 + sigma_i^2) against the oracle: the dense
definition at sizes it handles, the state-space recursion with per-step
variances at n = 2^20.  Bars as for scalar noise: log det within 1e-10
relative, residual ||y - C x|| / ||y|| within 1e-10 (FP64 factor); the mixed
factor's refined solve to its 1e-10 residual target."""
import numpy as np
import pytest

import oracle
import paper_1403_6015_amd as H
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _noise(n, seed, lo=0.01, hi=0.5):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def _check(p, nz, opts_kw=None, res_tol=1e-10):
    kw = dict(opts_kw or {})
    opts = H.Opts(noise=nz, **kw)
    announce("noise %s kernel=%d n=%d dim=%d %s" % (p.name, p.kernel, p.n, p.dim, kw))
    ref = oracle.gp_dense_noise(p.x, p.y, p.kernel, p.theta, p.sigma2, nz)
    f = H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, opts)
    ld = f.logdet()
    alpha = f.solve(p.y)
    f.free()
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    C[np.diag_indices(p.n)] += nz
    res = np.linalg.norm(p.y - C @ alpha) / np.linalg.norm(p.y)
    rel = abs(ld - ref["logdet"]) / abs(ref["logdet"])
    print("logdet rel %.2e residual %.2e" % (rel, res))
    assert rel <= 1e-10
    assert res <= res_tol
    ll, ld2, q = H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, opts)
    assert abs(ld2 - ref["logdet"]) <= 1e-10 * abs(ref["logdet"])
    assert abs(ll - ref["loglik"]) <= 1e-9 * abs(ref["loglik"])
    assert abs(q - ref["quad"]) <= 1e-9 * abs(ref["quad"])


def test_matern_heteroscedastic():
    p = wl.matern1d(4096)
    _check(p, _noise(p.n, 1))


def test_two_dimensional_heteroscedastic():
    p = wl.random_problem(2000, 2, wl.K_SE, seed=14, ell=0.6, sigma2=0.1, leaf=100, tol=1e-13)
    _check(p, _noise(p.n, 2), dict(max_rank=64))


def test_mixed_factor_with_noise():
    p = wl.matern1d(4096)
    _check(p, _noise(p.n, 3), dict(precision=H.MIXED))


def test_uniform_variances_equal_scalar_noise():
    p = wl.matern1d(4096)
    c = 0.2
    announce("uniform noise n=%d" % p.n)
    a = H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, p.leaf, p.tol,
                    H.Opts(noise=np.full(p.n, c)))
    b = H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2 + c, p.leaf, p.tol)
    assert np.allclose(a, b, rtol=1e-13, atol=0)


def test_full_size_against_kalman():
    p = wl.matern1d()
    nz = _noise(p.n, 4)
    announce("noise full size n=%d" % p.n)
    ll, ld, q = H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, p.leaf, p.tol,
                            H.Opts(noise=nz, presorted=1))
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, want_alpha=False, noise=nz)
    print("full size: logdet rel %.2e quad rel %.2e" % (abs(ld - kf["logdet"]) / abs(kf["logdet"]),
                                                        abs(q - kf["quad"]) / abs(kf["quad"])))
    assert abs(ld - kf["logdet"]) <= 1e-10 * abs(kf["logdet"])
    assert abs(q - kf["quad"]) <= 1e-9 * abs(kf["quad"])
    assert abs(ll - kf["loglik"]) <= 1e-9 * abs(kf["loglik"])


def test_prediction_through_a_noisy_factor():
    p = wl.matern1d(4096)
    nz = _noise(p.n, 5)
    xt = np.array([[0.0], [1.3], [2.0], [3.9], [4.5]])
    announce("noise predict n=%d" % p.n)
    f = H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, H.Opts(noise=nz))
    mean, var = f.predict(p.y, xt)
    f.free()
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    C[np.diag_indices(p.n)] += nz
    G = oracle.cholesky(C)
    Ks = oracle.cross_matrix(xt, p.x, p.kernel, p.theta)
    rmean = Ks @ oracle.chol_solve(G, p.y)
    rvar = np.array([p.theta[0] ** 2 - Ks[j] @ oracle.chol_solve(G, Ks[j])
                     for j in range(len(xt))])
    assert np.max(np.abs(mean - rmean)) <= 1e-9 * max(1.0, np.max(np.abs(rmean)))
    assert np.max(np.abs(var - rvar)) <= 1e-9
