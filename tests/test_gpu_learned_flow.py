"""End-to-end surrogate-screened sampling on a small GP (n = 8192): the
network trained on exact HODLR likelihoods predicts held-out likelihoods to
within a nat, delayed acceptance spends fewer exact evaluations per effective
sample than plain Metropolis with the same proposal, and both chains agree on
the posterior mean within Monte Carlo error."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def test_surrogate_screened_sampling_gains_over_plain_mh():
    from paper_1403_6015_amd import learned as LR
    n = 8192
    announce("learned flow n=%d" % n)
    p = wl.learned(n)
    gp = LR.ExactGP(p.x, p.y, kernel=p.kernel, leaf=p.leaf, tol=p.tol, max_rank=16, chunk=256)
    t_true = np.log([p.theta[0], p.theta[1], p.sigma2])
    mode, cov = LR.laplace(gp, t_true, 0.1)
    # the exact likelihood at the mode agrees with the Kalman oracle
    a, ell, s2 = np.exp(mode)
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, (a, ell), s2, want_alpha=False)
    assert abs(gp.loglik(mode[None])[0] - kf["loglik"]) <= 1e-9 * abs(kf["loglik"])
    X, T = LR.training_set(gp, mode, cov, n=3000)
    sur = LR.Surrogate(seed=1)
    hist = sur.fit(X[500:], T[500:], epochs=120, batch=128, lr=2e-3)
    assert hist[-20:].mean() < 0.05 * hist[:20].mean()
    # accuracy where the walkers live: held-out points within 15 nats of the mode
    rmse, nb = LR.bulk_rmse(sur.predict(X[:500]), T[:500], gp.loglik(mode[None])[0])
    assert nb >= 100 and rmse < 1.0, (rmse, nb)
    sd = np.sqrt(np.diag(cov))
    lo, hi = mode - 12 * sd, mode + 12 * sd
    W, steps, burn = 32, 160, 40
    rng = np.random.default_rng(2)
    start = np.clip(mode + rng.standard_normal((W, 3)) @ np.linalg.cholesky(cov).T, lo, hi)
    chol = 2.38 / np.sqrt(3.0) * np.linalg.cholesky(cov)
    out = {}
    for name, s in (("plain", None), ("delayed", sur)):
        chain, tal, secs = LR.sample(gp, start, chol, lo, hi, steps, surrogate=s, seed=3,
                                     block=40)
        post = chain[burn:]
        out[name] = dict(tal=tal, ess=LR.chain_ess(chain, burn), mean=post.reshape(-1, 3).mean(0),
                         var=post.reshape(-1, 3).var(0))
    pl, da = out["plain"], out["delayed"]
    assert da["tal"]["exact_evals"] < 0.7 * pl["tal"]["exact_evals"]
    assert da["tal"]["accepted"] > 0.5 * da["tal"]["survivors"]   # stage 2 rarely overrules
    assert da["ess"] / da["tal"]["exact_evals"] > pl["ess"] / pl["tal"]["exact_evals"]
    se = np.sqrt(pl["var"] / pl["ess"] + da["var"] / da["ess"])
    assert np.all(np.abs(da["mean"] - pl["mean"]) <= 5 * se), (da["mean"], pl["mean"], se)
