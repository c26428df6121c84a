"""GPU tests of speculative plan calls (hodlr_opts.speculate = 1): gp_loglik_dev
assumes the previous call's panel widths and large-block step count instead
of waiting for the compression's statistics, and a device check decides
whether the call stands or is redone the ordinary way.

* The same likelihood twice: the second call runs speculatively
  (hodlr_plan_info speculated = 1) and its outputs and C^{-1} y are
  bit-identical to the first call's and to a plan without speculation.
* A call whose ranks exceed the previous widths (a shorter length scale after
  a longer one): the check misses, the call is redone and equals the plan
  without speculation bit for bit; speculated = 0; the next call on the same
  parameters speculates again.
* A call whose ranks fit inside wider previous widths (a longer length scale
  after a shorter one): speculative, within 1e-13 of the plan without
  speculation (zero padding columns change the rounding of the coupling
  solves only).
* The 1-D Matern workload at n = 2^20 twice: the second call speculative and
  bit-identical to the first, log det within 1e-10 of the Kalman oracle.
* The option is validated (EINVAL outside {0, 1}).
"""
import numpy as np
import pytest

import oracle
import paper_1403_6015_amd as H
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


class DevCase:
    """One problem's device arrays and a plan with the given speculation."""

    def __init__(self, p, speculate):
        import torch
        self.p = p
        dev = torch.device("cuda:0")
        perm = H.hodlr_order(p.x, p.leaf)
        xo, yo = p.x[perm], p.y[perm]
        self.opts = H.Opts(max_rank=64, presorted=1, speculate=speculate)
        self.plan = H.Plan(p.n, p.dim, p.leaf, self.opts)
        self.d_x = torch.from_numpy(np.ascontiguousarray(xo.T)).to(dev)
        self.d_y = torch.from_numpy(np.ascontiguousarray(yo)).to(dev)
        nb = self.plan.workspace_bytes
        self.work = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.out = torch.zeros(8, dtype=torch.float64, device=dev)
        self.z = torch.zeros(p.n, dtype=torch.float64, device=dev)

    def call(self, theta=None, sigma2=None):
        import torch
        p = self.p
        H.gp_loglik_dev(self.plan, self.d_x, p.kernel, theta or p.theta,
                        p.sigma2 if sigma2 is None else sigma2, self.d_y, p.tol, self.work,
                        self.plan.workspace_bytes, None, self.out, self.z)
        torch.cuda.synchronize()
        return self.out.cpu().numpy()[:3].copy(), self.z.cpu().numpy().copy(), self.plan.info()


def test_same_likelihood_twice_is_speculative_and_bit_identical():
    p = wl.random_problem(8192, 1, wl.K_SE, 611, ell=0.02, sigma2=0.02, leaf=64, tol=1e-10)
    announce("speculation: same likelihood twice, 1-D SE n=%d" % p.n)
    s = DevCase(p, 1)
    o1, z1, i1 = s.call()
    o2, z2, i2 = s.call()
    r = DevCase(p, 0)
    o0, z0, _ = r.call()
    print("  ranks %s, speculated %d then %d" % (i2["rank_max"], i1["speculated"], i2["speculated"]),
          flush=True)
    assert i1["speculated"] == 0 and i2["speculated"] == 1
    assert i2["rank_max"] == i1["rank_max"]
    assert np.array_equal(o1, o2) and np.array_equal(z1, z2)
    assert np.array_equal(o0, o2) and np.array_equal(z0, z2)


def test_ranks_above_the_widths_are_redone():
    p = wl.random_problem(8192, 1, wl.K_SE, 612, ell=0.05, sigma2=0.02, leaf=64, tol=1e-10)
    announce("speculation: ranks grow (l 0.05 -> 0.01), 1-D SE n=%d" % p.n)
    s = DevCase(p, 1)
    _, _, ia = s.call()
    short = (1.0, 0.01)
    o, z, ib = s.call(theta=short)
    r = DevCase(p, 0)
    o0, z0, i0 = r.call(theta=short)
    print("  ranks l=0.05 %s; l=0.01 %s; speculated %d" % (ia["rank_max"], ib["rank_max"],
                                                          ib["speculated"]), flush=True)
    assert any(b > a for a, b in zip(ia["rank_max"], ib["rank_max"]))
    assert ib["speculated"] == 0
    assert ib["rank_max"] == i0["rank_max"]
    assert np.array_equal(o, o0) and np.array_equal(z, z0)
    o2, z2, ic = s.call(theta=short)
    assert ic["speculated"] == 1
    assert np.array_equal(o2, o0) and np.array_equal(z2, z0)


def test_ranks_inside_wider_widths_stay_speculative():
    p = wl.random_problem(8192, 1, wl.K_SE, 613, ell=0.01, sigma2=0.02, leaf=64, tol=1e-10)
    announce("speculation: ranks shrink (l 0.01 -> 0.012), 1-D SE n=%d" % p.n)
    s = DevCase(p, 1)
    _, _, ia = s.call()
    longer = (1.0, 0.012)
    o, z, ib = s.call(theta=longer)
    r = DevCase(p, 0)
    o0, z0, i0 = r.call(theta=longer)
    print("  ranks l=0.01 %s; l=0.012 %s; speculated %d" % (ia["rank_max"], ib["rank_max"],
                                                           ib["speculated"]), flush=True)
    assert ib["rank_max"] == i0["rank_max"]
    if ib["speculated"] == 1:
        assert all(b <= a for a, b in zip(ia["rank_max"], ib["rank_max"]))
    for j in range(3):
        assert abs(o[j] - o0[j]) <= 1e-13 * abs(o0[j]), j
    assert np.max(np.abs(z - z0)) <= 1e-12 * np.max(np.abs(z0))


def test_full_size_matern_twice():
    p = wl.matern1d(1 << 20)
    announce("speculation: 1-D Matern n=2^20 twice")
    s = DevCase(p, 1)
    o1, z1, i1 = s.call()
    o2, z2, i2 = s.call()
    assert i2["speculated"] == 1
    assert np.array_equal(o1, o2) and np.array_equal(z1, z2)
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, want_alpha=False)
    assert abs(o2[1] - kf["logdet"]) <= 1e-10 * abs(kf["logdet"])


def test_option_is_validated():
    with pytest.raises(H.HodlrError) as ei:
        H.Plan(4096, 1, 64, H.Opts(speculate=2))
    assert ei.value.name == "EINVAL"
