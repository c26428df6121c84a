"""Metropolis-Hastings and delayed-acceptance steps, written plainly (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's outer loop (§1, Eq. (1) and the posterior over hyperparameters
that it feeds) draws hyperparameters from p(theta | y), proportional to
exp(l(theta)) p(theta).  One random-walk Metropolis step per walker:

    theta' = theta + L eps                   (eps ~ N(0, I), L lower-triangular)
    accept if log u < log pi(theta') - log pi(theta).

Delayed acceptance (Christen and Fox, 2005) screens the proposal first with a
cheap approximation pi~ and evaluates pi only for proposals that survive:

    stage 1: accept if log u1 < log pi~(theta') - log pi~(theta)
    stage 2: accept if log u2 < [log pi(theta') - log pi(theta)]
                                 - [log pi~(theta') - log pi~(theta)]

The second stage makes the chain reversible with respect to pi for any pi~
(the surrogate only changes efficiency).  Both pi and pi~ include the same
log-prior, so the prior cancels in the stage-2 ratio.  The random numbers
(eps, u1, u2) are inputs here, as they are to the device kernels.

The prior is uniform on a box in log theta (log a, log l, log sigma^2); a
proposal outside the box has log pi = -inf and is rejected at stage 1 without
any likelihood evaluation.
"""
from __future__ import annotations

import numpy as np


def in_box(lt, lo, hi):
    lt = np.atleast_2d(lt)
    return np.all((lt >= lo) & (lt <= hi), axis=1)


def propose(theta, chol, eps):
    """theta' = theta + eps L^T row by row (theta, eps: [W, 3])."""
    return np.asarray(theta) + np.asarray(eps) @ np.asarray(chol).T


def mh_step(theta, lp, prop, lp_prop, u, lo, hi):
    """Plain MH decision; lp are log-likelihoods (prior uniform on the box).
    Returns (new theta, new lp, accepted mask)."""
    ok = in_box(prop, lo, hi)
    acc = ok & (np.log(u) < (lp_prop - lp))
    return (np.where(acc[:, None], prop, theta), np.where(acc, lp_prop, lp), acc)


def da_stage1(sur, sur_prop, prop, u1, lo, hi):
    """Stage-1 survivors (mask) from surrogate values at theta and theta'."""
    ok = in_box(prop, lo, hi)
    return ok & (np.log(u1) < (sur_prop - sur))


def da_stage2(theta, lp, sur, prop, lp_prop, sur_prop, survivors, u2):
    """Stage-2 decision for the survivors; lp_prop only matters where
    survivors is True.  Returns (theta, lp, sur, accepted mask)."""
    lp_prop = np.where(survivors, lp_prop, 0.0)
    ratio = (lp_prop - lp) - (sur_prop - sur)
    acc = survivors & (np.log(u2) < ratio)
    return (np.where(acc[:, None], prop, theta), np.where(acc, lp_prop, lp),
            np.where(acc, sur_prop, sur), acc)


def autocorr_ess(chain):
    """Effective sample size of a scalar chain by Geyer's initial positive
    sequence: ESS = N / (1 + 2 sum rho_k), summing autocorrelation pairs
    (rho_{2m} + rho_{2m+1}) while they stay positive."""
    x = np.asarray(chain, dtype=np.float64)
    n = x.size
    x = x - x.mean()
    var = np.dot(x, x) / n
    if var == 0.0:
        return float(n)
    f = np.fft.rfft(x, 2 * n)
    ac = np.fft.irfft(f * np.conj(f))[:n] / (n * var)
    s = 0.0
    m = 0
    while 2 * m + 1 < n:
        pair = ac[2 * m] + ac[2 * m + 1]
        if pair <= 0.0:
            break
        s += pair
        m += 1
    tau = -1.0 + 2.0 * s
    return float(n / max(tau, 1e-12))
