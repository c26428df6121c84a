"""GPU parity of the log-likelihood gradient (gp_loglik_grad_dev: central
differences of 7 likelihoods, the two sigma^2 items on the point's
compression).

* Every component against the dense analytic gradient of the oracle
  (1/2 alpha^T C_p alpha - 1/2 tr(C^{-1} C_p)), for every kernel in 1-D and the
  squared exponential in 2-D.  The bar is 1e-6 (|L| / p + |dL/dp|) per
  component p: the difference's truncation error is about
  rel_step^2 / 6 |L| / p (1.7e-9 |L| / p at the default 1e-4) and its
  rounding about eps_L |L| / (2 rel_step p) for a likelihood correct to eps_L
  relative (~1e-12 here: 5e-9 |L| / p).
* At the Matern-3/2 workload's full size (n = 2^20), against the same central
  difference of the exact O(n) Kalman likelihood at the same seven parameter
  points: only the factorization's own error differs, bar 1e-7 |L| / p.
* The value part equals gp_loglik_dev's, and bad arguments are rejected.
"""
import numpy as np
import pytest

import oracle
from oracle import grad_ref
import paper_1403_6015_amd as H
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _dev_grad(p, opts, rel_step=0.0, presorted=False):
    import torch
    dev = torch.device("cuda:0")
    if presorted:
        xo, yo = p.x, p.y
    else:
        perm = H.hodlr_order(p.x, p.leaf)
        xo, yo = p.x[perm], p.y[perm]
    plan = H.Plan(p.n, p.dim, p.leaf, opts)
    d_x = torch.from_numpy(np.ascontiguousarray(xo.T)).to(dev)
    d_y = torch.from_numpy(np.ascontiguousarray(yo)).to(dev)
    nb = plan.grad_workspace_bytes
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    out = torch.full((6,), float("nan"), dtype=torch.float64, device=dev)
    H.gp_loglik_grad_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, rel_step, work, nb,
                         None, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    w1 = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    o1 = torch.zeros(8, dtype=torch.float64, device=dev)
    H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, w1, plan.workspace_bytes,
                    None, o1)
    torch.cuda.synchronize()
    return o, o1.cpu().numpy()[:3], plan


CASES = [
    ("se1d", lambda: wl.random_problem(2048, 1, wl.K_SE, 301, ell=0.05, sigma2=0.02, leaf=64,
                                       tol=1e-12)),
    ("matern1d", lambda: wl.random_problem(2048, 1, wl.K_MATERN32, 302, ell=0.1, sigma2=0.05,
                                           leaf=64, tol=1e-12)),
    ("exp1d", lambda: wl.random_problem(2048, 1, wl.K_EXP, 303, ell=0.2, sigma2=0.05, leaf=64,
                                        tol=1e-12)),
    ("imq1d", lambda: wl.random_problem(2048, 1, wl.K_IMQ, 304, ell=0.05, sigma2=0.05, leaf=64,
                                        tol=1e-12)),
    ("se2d", lambda: wl.random_problem(3000, 2, wl.K_SE, 305, ell=0.1, sigma2=0.02, leaf=128,
                                       tol=1e-12)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_gradient_matches_dense_analytic_gradient(name, make):
    p = make()
    announce("gradient %s n=%d dim=%d" % (name, p.n, p.dim))
    o, single, _ = _dev_grad(p, H.Opts(max_rank=256))
    ref = grad_ref.gp_dense_grad(p.x, p.y, p.kernel, p.theta, p.sigma2)
    L = ref["loglik"]
    pars = [p.theta[0], p.theta[1], p.sigma2]
    assert abs(o[0] - single[0]) <= 1e-12 * abs(single[0])
    assert abs(o[0] - L) <= 1e-10 * abs(L)
    for j in range(3):
        g, gr = o[3 + j], ref["grad"][j]
        bar = 1e-6 * (abs(L) / pars[j] + abs(gr))
        print("  %s dL/dp%d: %.10e ref %.10e  err %.2e  bar %.2e" % (name, j, g, gr, abs(g - gr), bar),
              flush=True)
        assert abs(g - gr) <= bar, (j, g, gr)


def test_mixed_plan_gradient():
    p = CASES[1][1]()
    announce("gradient mixed plan n=%d" % p.n)
    o, _, _ = _dev_grad(p, H.Opts(max_rank=256, precision=H.MIXED))
    ref = grad_ref.gp_dense_grad(p.x, p.y, p.kernel, p.theta, p.sigma2)
    pars = [p.theta[0], p.theta[1], p.sigma2]
    for j in range(3):
        bar = 1e-5 * (abs(ref["loglik"]) / pars[j] + abs(ref["grad"][j]))
        assert abs(o[3 + j] - ref["grad"][j]) <= bar, j


def test_full_size_matern_against_kalman_difference():
    p = wl.matern1d(1 << 20)
    announce("gradient matern n=2^20 against the Kalman difference")
    o, single, _ = _dev_grad(p, H.Opts(max_rank=64, presorted=1), presorted=True)
    base = [p.theta[0], p.theta[1], p.sigma2]
    h = 1e-4
    L0 = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, want_alpha=False)["loglik"]
    assert abs(o[0] - L0) <= 1e-10 * abs(L0)
    for j in range(3):
        up, dn = list(base), list(base)
        up[j] = base[j] * (1.0 + h)
        dn[j] = base[j] * (1.0 - h)
        Lu = oracle.kalman_matern32(p.x[:, 0], p.y, up[:2], up[2], want_alpha=False)["loglik"]
        Ld = oracle.kalman_matern32(p.x[:, 0], p.y, dn[:2], dn[2], want_alpha=False)["loglik"]
        gk = (Lu - Ld) / (up[j] - dn[j])
        bar = 1e-7 * abs(L0) / base[j]
        print("  n=2^20 dL/dp%d: %.10e Kalman difference %.10e err %.2e bar %.2e"
              % (j, o[3 + j], gk, abs(o[3 + j] - gk), bar), flush=True)
        assert abs(o[3 + j] - gk) <= bar, j


def test_gradient_rejects_bad_arguments():
    import torch
    p = CASES[0][1]()
    plan = H.Plan(p.n, 1, p.leaf, H.Opts(max_rank=64, presorted=1))
    dev = torch.device("cuda:0")
    d_x = torch.from_numpy(np.ascontiguousarray(p.x.T)).to(dev)
    d_y = torch.from_numpy(p.y).to(dev)
    nb = plan.grad_workspace_bytes
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    out = torch.zeros(6, dtype=torch.float64, device=dev)
    for kw in (dict(sigma2=0.0), dict(rel_step=0.5), dict(nb=nb - 1), dict(theta=(1.0, -0.1))):
        args = dict(theta=p.theta, sigma2=p.sigma2, rel_step=0.0, nb=nb)
        args.update(kw)
        with pytest.raises(H.HodlrError) as ei:
            H.gp_loglik_grad_dev(plan, d_x, p.kernel, args["theta"], args["sigma2"], d_y, p.tol,
                                 args["rel_step"], work, args["nb"], None, out)
        assert ei.value.name == "EINVAL", kw
