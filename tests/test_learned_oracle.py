"""Pins of the surrogate-network and sampler oracles against what the
mathematics fixes: central finite differences for the gradient, closed forms
for degenerate networks and for Adam's first step, the exact autocorrelation
time of an AR(1) process for the effective-sample-size estimator, and the
stationary moments of a Gaussian target for delayed acceptance (with a
planted mistake showing the check discriminates)."""
import numpy as np
import pytest

from oracle import mcmc_ref as mc
from oracle import mlp_ref as mr

NORM = {"mu_in": np.array([0.1, -0.3, 0.2]), "sd_in": np.array([0.5, 1.5, 0.8]),
        "mu_out": 3.0, "sd_out": 2.5}


def test_parameter_count():
    assert mr.NPARAM == 17153


def test_bf16_rounding_is_nearest_even():
    one = 1.0
    assert mr.bf16_round(one) == 1.0
    assert mr.bf16_round(1.0 + 2.0 ** -8) == 1.0                    # tie -> even (down)
    assert mr.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6    # tie -> even (up)
    assert mr.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert mr.bf16_round(-1.0 - 2.0 ** -8 - 2.0 ** -20) == -(1.0 + 2.0 ** -7)
    x = np.random.default_rng(1).standard_normal(1000)
    r = mr.bf16_round(x)
    # 8 significant bits: unit roundoff 2^-8
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))
    assert np.any(np.abs(r - x) > 2.0 ** -10 * np.abs(x))


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    p = mr.init_params(5) + 0.05 * rng.standard_normal(mr.NPARAM)
    X = rng.normal(size=(7, 3))
    T = rng.normal(3.0, 4.0, size=7)
    loss, g = mr.loss_and_grad(p, X, T, NORM)
    idx = np.concatenate([rng.choice(mr.NPARAM, 60, replace=False), [mr.NPARAM - 1, 0, 383, 384]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mr.NPARAM)
        e[k] = h
        fd = (mr.loss_and_grad(p + e, X, T, NORM)[0] - mr.loss_and_grad(p - e, X, T, NORM)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_zero_network_outputs_the_head_bias():
    p = np.zeros(mr.NPARAM)
    p[-1] = 0.75
    out, _ = mr.forward(p, np.random.default_rng(0).normal(size=(5, 3)), NORM)
    assert np.allclose(out, NORM["mu_out"] + NORM["sd_out"] * 0.75, rtol=0, atol=1e-15)


def test_small_weights_reduce_to_the_linear_composition():
    rng = np.random.default_rng(4)
    eps = 1e-4
    P = mr.unpack(eps * rng.standard_normal(mr.NPARAM))
    P["b1"][:] = 0
    P["b2"][:] = 0
    P["b3"][:] = 0
    p = np.concatenate([P[n].ravel() for n, _ in mr.SIZES])
    X = rng.normal(size=(4, 3))
    U = (X - NORM["mu_in"]) / NORM["sd_in"]
    lin = U @ (P["W3"] @ P["W2"] @ P["W1"])
    out, _ = mr.forward(p, X, NORM)
    o = (out - NORM["mu_out"]) / NORM["sd_out"]
    # tanh(z) = z - z^3/3 + ...: relative deviation O(eps^2)
    assert np.allclose(o, lin, rtol=1e-6, atol=0)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(6)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = mr.adam_step(p, np.zeros(50), np.zeros(50), g, 1, 0.01)
    # mhat = g and vhat = g^2 at t = 1
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_minimizes_a_quadratic():
    c = np.linspace(-2, 2, 9)
    p = np.zeros(9)
    m = np.zeros(9)
    v = np.zeros(9)
    for t in range(1, 3001):
        p, m, v = mr.adam_step(p, m, v, p - c, t, 0.01)
    assert np.max(np.abs(p - c)) < 1e-3


def test_ess_of_iid_and_ar1():
    rng = np.random.default_rng(8)
    n = 200_000
    iid = rng.standard_normal(n)
    assert 0.9 * n <= mc.autocorr_ess(iid) <= 1.1 * n
    rho = 0.9
    z = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = z[0] / np.sqrt(1 - rho * rho)
    for i in range(1, n):
        x[i] = rho * x[i - 1] + z[i]
    # integrated autocorrelation time of AR(1): (1 + rho) / (1 - rho)
    expect = n * (1 - rho) / (1 + rho)
    assert 0.85 * expect <= mc.autocorr_ess(x) <= 1.15 * expect


def _gauss_chain(W, steps, seed, surrogate, mistake=False):
    rng = np.random.default_rng(seed)
    lo, hi = np.full(3, -10.0), np.full(3, 10.0)
    L = 1.0 * np.eye(3)

    def lp(t):
        return -0.5 * np.sum(t * t, axis=1)

    th = rng.normal(size=(W, 3))
    l0 = lp(th)
    s0 = surrogate(th)
    draws = []
    exact_evals = 0
    for _ in range(steps):
        eps = rng.standard_normal((W, 3))
        u1 = rng.uniform(size=W)
        u2 = rng.uniform(size=W)
        prop = mc.propose(th, L, eps)
        sp = surrogate(prop)
        surv = mc.da_stage1(s0, sp, prop, u1, lo, hi)
        exact_evals += int(surv.sum())
        lpp = np.where(surv, lp(prop), np.nan)
        if mistake:   # planted: stage 2 without the surrogate correction
            th, l0, s0, _ = mc.da_stage2(th, l0, np.zeros(W), prop, lpp, np.zeros(W), surv, u2)
            s0 = surrogate(th)
        else:
            th, l0, s0, _ = mc.da_stage2(th, l0, s0, prop, lpp, sp, surv, u2)
        draws.append(th.copy())
    return np.array(draws[steps // 5:]).reshape(-1, 3), exact_evals


def test_delayed_acceptance_keeps_the_exact_target():
    def biased(t):
        return -0.5 * np.sum((t - 0.7) ** 2, axis=1) / 1.5 ** 2

    d, ev = _gauss_chain(256, 3000, 11, biased)
    assert np.all(np.abs(d.mean(axis=0)) < 0.03), d.mean(axis=0)
    assert np.all(np.abs(d.var(axis=0) - 1.0) < 0.05), d.var(axis=0)
    assert ev < 256 * 3000   # the screen saved exact evaluations
    bad, _ = _gauss_chain(256, 3000, 11, biased, mistake=True)
    assert np.all(bad.mean(axis=0) > 0.1), bad.mean(axis=0)


def test_perfect_surrogate_reduces_to_plain_mh():
    rng = np.random.default_rng(12)
    W = 64
    lo, hi = np.full(3, -3.0), np.full(3, 3.0)
    th = rng.normal(size=(W, 3))
    lp = -0.5 * np.sum(th * th, axis=1)
    eps = rng.standard_normal((W, 3))
    u1 = rng.uniform(size=W)
    u2 = rng.uniform(size=W)
    prop = mc.propose(th, 0.8 * np.eye(3), eps)
    lpp = -0.5 * np.sum(prop * prop, axis=1)
    t_mh, l_mh, acc_mh = mc.mh_step(th, lp, prop, lpp, u1, lo, hi)
    surv = mc.da_stage1(lp, lpp, prop, u1, lo, hi)
    t_da, l_da, _, acc_da = mc.da_stage2(th, lp, lp, prop, lpp, lpp, surv, u2)
    assert np.array_equal(acc_mh, acc_da)
    assert np.array_equal(t_mh, t_da) and np.array_equal(l_mh, l_da)


def test_proposal_applies_the_lower_factor_not_its_transpose():
    """theta' = theta + L eps with a non-diagonal lower-triangular L: a unit
    eps_k moves theta along column k of L, and over many draws the increments
    have covariance L L^T (an L / L^T mix-up gives L^T L, which differs here)."""
    L = np.array([[0.5, 0.0, 0.0], [0.3, 0.4, 0.0], [-0.2, 0.6, 0.7]])
    assert not np.allclose(L @ L.T, L.T @ L)
    th = np.array([[0.1, -0.2, 0.3]])
    for k in range(3):
        e = np.zeros((1, 3))
        e[0, k] = 1.0
        assert np.array_equal(mc.propose(np.zeros((1, 3)), L, e)[0], L[:, k]), k
        step = mc.propose(th, L, e) - th
        assert np.allclose(step[0], L[:, k], rtol=0, atol=1e-15), (k, step, L[:, k])
    rng = np.random.default_rng(21)
    N = 400000
    eps = rng.standard_normal((N, 3))
    inc = mc.propose(np.zeros((N, 3)), L, eps)
    cov = inc.T @ inc / N
    # Monte Carlo error of each covariance entry ~ sqrt(2 / N) * scale ~ 2e-3
    assert np.max(np.abs(cov - L @ L.T)) < 1e-2, cov
    assert np.max(np.abs(cov - L.T @ L)) > 0.1


def _term_magnitudes(p, X, T):
    """Per gradient entry: the sum of |terms| of the sums that form it and the
    largest single |term| (chain rule of ``loss_and_grad`` with absolute
    values)."""
    P = mr.unpack(p)
    _, c = mr.forward(p, X, NORM)
    B = X.shape[0]
    go = 2.0 * (c["O"] - (T - NORM["mu_out"]) / NORM["sd_out"]) / B
    ad = np.abs(go[:, None] * P["W3"][None, :] * (1 - c["H2"] ** 2))
    mz1 = (ad @ np.abs(P["W2"])) * (1 - c["H1"] ** 2)
    aU, aH1, aH2, ag = np.abs(c["U"]), np.abs(c["H1"]), np.abs(c["H2"]), np.abs(go)
    mag = np.concatenate([(mz1.T @ aU).ravel(), mz1.sum(0), (ad.T @ aH1).ravel(), ad.sum(0),
                          aH2.T @ ag, [ag.sum()]])
    return mag


def test_bf16_operand_gradient_stays_within_the_rounding_bound():
    """With the operands of the two 128-wide products rounded to BF16, every
    gradient entry moves by at most a few BF16 unit roundoffs of the summed
    term magnitudes (first-order propagation of relative 2^-8 perturbations
    of h1 and dz2 through two products), and does move (the rounding is
    applied)."""
    rng = np.random.default_rng(8)
    p = mr.bf16_round(mr.init_params(8) + 0.05 * rng.standard_normal(mr.NPARAM))
    X = rng.normal(size=(50, 3))
    T = rng.normal(3.0, 4.0, size=50)
    l0, g0 = mr.loss_and_grad(p, X, T, NORM)
    l1, g1 = mr.loss_and_grad(p, X, T, NORM, bf16_products=True)
    mag = _term_magnitudes(p, X, T)
    d = np.abs(g1 - g0)
    assert np.all(d <= 6 * 2.0 ** -8 * mag + 1e-15), np.max(d / (mag + 1e-300))
    assert np.max(d / (mag + 1e-300)) > 2.0 ** -14
    assert abs(l1 - l0) <= 4 * 2.0 ** -8 * max(l0, 1e-12)
    # the default is the exact chain rule
    assert np.array_equal(mr.loss_and_grad(p, X, T, NORM, bf16_products=False)[1], g0)
