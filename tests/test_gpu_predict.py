"""GPU parity of prediction through the factor (§2.1: predictive mean
k(xt, x) C^{-1} y and variance k(xt, xt) - k(xt, x) C^{-1} k(x, xt)) against
the dense oracle at sizes it handles, against the exact O(n) Kalman solves
for Matern-3/2 at n = 2^20, and against the constant-kernel closed form.
Bars: mean within 1e-9 of max(1, max |mean|), variance within 1e-9 a^2 (FP64
factor); 1e-8 for the mixed factor, whose solves are refined to 1e-10."""
import numpy as np
import pytest

import oracle
import paper_1403_6015_amd as H
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _test_points(x, m, seed):
    """New inputs: some exactly on training points, some between them, some
    outside the data's range (per coordinate), one repeated."""
    rng = np.random.default_rng(seed)
    lo, hi = x.min(axis=0), x.max(axis=0)
    span = hi - lo
    on = x[rng.choice(len(x), m // 4, replace=False)]
    inside = lo + rng.uniform(0, 1, (m // 2, x.shape[1])) * span
    outside = lo + rng.uniform(-0.2, 1.2, (m - m // 4 - m // 2 - 1, x.shape[1])) * span
    return np.vstack([on, inside, outside, on[:1]])


def _check(p, opts=None, m=64, tol=1e-9):
    xt = _test_points(p.x, m, seed=p.n)
    announce("predict %s kernel=%d n=%d dim=%d m=%d" % (p.name, p.kernel, p.n, p.dim, len(xt)))
    f = H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, opts)
    mean, var = f.predict(p.y, xt)
    f.free()
    rmean, rvar = oracle.gp_predict_dense(p.x, p.y, xt, p.kernel, p.theta, p.sigma2)
    a2 = p.theta[0] ** 2
    em = np.max(np.abs(mean - rmean)) / max(1.0, np.max(np.abs(rmean)))
    ev = np.max(np.abs(var - rvar)) / a2
    print("mean err %.2e var err %.2e" % (em, ev))
    assert em <= tol, em
    assert ev <= tol, ev
    assert np.all(var >= -tol * a2)


def test_matern_slice():
    _check(wl.matern1d(4096))


def test_se_small():
    _check(wl.se1d_small())


def test_two_dimensional():
    # the 2-D configuration the likelihood parity holds to the 1e-10 residual
    # bar (one application of an FP64 factor is accurate to about
    # tol ||K|| / sigma^2)
    _check(wl.random_problem(3000, 2, wl.K_SE, seed=14, ell=0.6, sigma2=0.1, leaf=100,
                             tol=1e-13), H.Opts(max_rank=64))


def test_inverse_multiquadric():
    _check(wl.random_problem(3000, 1, wl.K_IMQ, seed=61, ell=0.1, sigma2=0.05, leaf=64,
                             tol=1e-12))


def test_mixed_factor_refined_solves():
    _check(wl.matern1d(4096), H.Opts(precision=H.MIXED), m=32, tol=1e-8)


def test_constant_kernel_closed_form():
    p = wl.rank1_points(1000)
    announce("predict constant kernel n=%d" % p.n)
    f = H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, p.leaf, p.tol)
    xt = np.array([[-1.0], [0.3], [5.0]])
    mean, var = f.predict(p.y, xt)
    f.free()
    a2, s2, n = p.theta[0] ** 2, p.sigma2, p.n
    assert mean == pytest.approx(np.full(3, a2 * p.y.sum() / (s2 + n * a2)), rel=1e-11)
    assert var == pytest.approx(np.full(3, a2 * s2 / (s2 + n * a2)), rel=1e-9)


def test_full_size_against_kalman():
    """n = 2^20: the mean at 8 new inputs from the exact alpha of the Kalman
    oracle and entry-by-entry kernel rows; the variance at 2 of them from
    the oracle's exact solves of C v = k(x, xt_j)."""
    p = wl.matern1d()
    xt = np.array([[0.0], [0.37], [123.456], [500.0], [p.x[777, 0]], [999.9], [1000.5],
                   [-4.0]])
    announce("predict full size n=%d m=%d" % (p.n, len(xt)))
    f = H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, p.leaf, p.tol)
    mean, _ = f.predict(p.y, xt, var=False)
    _, var2 = f.predict(p.y, xt[2:4])
    f.free()
    alpha = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2)["alpha"]
    Ks = oracle.cross_matrix(xt, p.x, p.kernel, p.theta)
    rmean = Ks @ alpha
    em = np.max(np.abs(mean - rmean)) / max(1.0, np.max(np.abs(rmean)))
    rvar = []
    for j in (2, 3):
        v = oracle.kalman_matern32(p.x[:, 0], Ks[j], p.theta, p.sigma2)["alpha"]
        rvar.append(p.theta[0] ** 2 - Ks[j] @ v)
    ev = np.max(np.abs(var2 - np.array(rvar)))
    print("full size: mean err %.2e var err %.2e" % (em, ev))
    assert em <= 1e-9
    assert ev <= 1e-9


def test_edges_and_errors():
    p = wl.matern1d(4096)
    announce("predict edges")
    f = H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, p.leaf, p.tol)
    mean, var = f.predict(p.y, np.zeros((0, 1)))
    assert mean.size == 0 and var.size == 0
    with pytest.raises(H.HodlrError) as e:
        f.predict(p.y, np.zeros((3, 2)))   # wrong dimension
    assert e.value.name == "EINVAL"
    with pytest.raises(H.HodlrError) as e:
        f.predict(p.y, np.array([[np.nan]]))
    assert e.value.name == "EINVAL"
    f.free()


def test_regression_rmse_follows_the_tolerance():
    """§5.6 experiment: the regression estimate K C^{-1} y at the 1024 data
    points of the synthetic model through the GPU factor; its RMSE differs
    from the dense oracle's by an amount proportional to the factorization
    precision, for smallest blocks of 20 and 64 points."""
    p = wl.regression_model()
    n = p.n
    exact, _ = oracle.gp_predict_dense(p.x, p.y, p.x, p.kernel, p.theta, p.sigma2, want_var=False)
    rm_exact = np.linalg.norm(p.y - exact) / np.sqrt(n)
    errs = {}
    for tol in (1e-4, 1e-7, 1e-10):
        for leaf in (20, 64):
            announce("regression tol=%g leaf=%d" % (tol, leaf))
            f = H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, leaf, tol)
            yh, _ = f.predict(p.y, p.x, var=False)
            f.free()
            d = abs(np.linalg.norm(p.y - yh) / np.sqrt(n) - rm_exact)
            e = np.max(np.abs(yh - exact))
            print("tol %g leaf %d: |dRMSE| %.2e, max |dy| %.2e" % (tol, leaf, d, e))
            assert d <= 1e-2 * tol + 1e-13
            assert e <= 10 * tol + 1e-11
            errs[tol, leaf] = e
    for leaf in (20, 64):
        assert errs[1e-4, leaf] > errs[1e-7, leaf] > errs[1e-10, leaf]
