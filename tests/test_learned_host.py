"""Host-side helpers of the sampling workflow: the product's ESS estimator
(Sokal windowing) against the AR(1) closed form and the oracle's
initial-positive-sequence estimator."""
import numpy as np

from oracle import mcmc_ref as mc
from paper_1403_6015_amd import learned as LR


def _ar1(rho, n, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = z[0] / np.sqrt(1 - rho * rho)
    for i in range(1, n):
        x[i] = rho * x[i - 1] + z[i]
    return x


def test_ess_matches_ar1_closed_form_and_oracle():
    for rho in (0.0, 0.5, 0.9):
        x = _ar1(rho, 100_000, 20 + int(10 * rho))
        expect = len(x) * (1 - rho) / (1 + rho)
        e = LR.ess(x)
        assert 0.85 * expect <= e <= 1.15 * expect, (rho, e, expect)
        assert abs(e - mc.autocorr_ess(x)) <= 0.15 * expect


def test_chain_ess_sums_walkers_and_takes_the_worst_coordinate():
    rng = np.random.default_rng(1)
    c = rng.standard_normal((4000, 3, 3))
    c[:, :, 2] = np.repeat(_ar1(0.9, 4000, 2)[:, None], 3, axis=1)
    tot = LR.chain_ess(c)
    one = LR.ess(c[:, 0, 2])
    assert abs(tot - 3 * one) <= 1e-9 * tot
