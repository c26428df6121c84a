"""One plan reused across hyperparameters whose cross-approximation ranks
differ: the large-block loop polls from the step where the previous call on
the plan finished, so this exercises polls that come too early and too late;
the results must equal those of a fresh plan bit for bit (the poll schedule
only decides when the host looks, not what is computed)."""
import numpy as np
import pytest

import paper_1403_6015_amd as H
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _call(plan, d_x, d_y, kernel, theta, sigma2, tol):
    import torch
    work = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    H.gp_loglik_dev(plan, d_x, kernel, theta, sigma2, d_y, tol, work, plan.workspace_bytes,
                    None, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:3]


def test_reused_plan_equals_fresh_plans_across_ranks():
    import torch
    p = wl.random_problem(32768, 1, wl.K_SE, seed=77, ell=1.0, sigma2=0.1, leaf=128, tol=1e-10,
                          lo=0.0, hi=20.0)
    announce("plan reuse SE n=%d" % p.n)
    # depths 0-2 hold the blocks with a side above 2048 (the polled loop):
    # their largest rank is 10 at l = 5 and 13 at l = 0.5
    ells = [5.0, 0.5, 5.0, 0.5, 0.05]
    big = [max(H.hodlr_build(p.x, p.kernel, (1.0, ell), p.sigma2, p.leaf, p.tol,
                             H.Opts(max_rank=64, presorted=1)).info()["rank_max"][:3])
           for ell in (5.0, 0.5)]
    assert big[0] != big[1], big   # the step counts really differ
    d_x = torch.from_numpy(np.ascontiguousarray(p.x.T)).cuda()
    d_y = torch.from_numpy(p.y.copy()).cuda()
    opts = H.Opts(max_rank=64, presorted=1)
    reused = H.Plan(p.n, 1, p.leaf, opts)
    for ell in ells:
        a = _call(reused, d_x, d_y, p.kernel, (1.0, ell), p.sigma2, p.tol)
        b = _call(H.Plan(p.n, 1, p.leaf, opts), d_x, d_y, p.kernel, (1.0, ell), p.sigma2, p.tol)
        assert np.all(np.isfinite(a)), (ell, a)
        assert np.array_equal(a, b), (ell, a, b)
