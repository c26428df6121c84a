"""GPU parity of the projected level form (hodlr_opts.level_form = 0, the
default for likelihoods): the bases' projections G = Z^T K^{-1} Z go up the
tree and C^{-1} y comes down it, with the coupling matrices and determinants
of the level-by-level factorization.

* Against the level-by-level form (level_form = 1) on the same plan and
  inputs, for every kernel in 1-D and for the squared exponential in 2-D:
  log det within 1e-12, the quadratic form within 1e-10 and C^{-1} y within
  1e-9 (relative; only the rounding order differs), and both against the dense
  oracle (log det 1e-10).
* The mixed form the same way (its FP32 panel is the leaf factor's only), with
  bars for the two forms' different FP32 roundings: log det 1e-8, the
  quadratic form 1e-6, the unrefined C^{-1} y 1e-4.
* Widths above the projected form's limits (2-D, ranks above 32) take the
  level-by-level form (info projected = 0) with unchanged results.
* The batched form (6 hyperparameter settings on shared points): every item
  against the Kalman oracle.
* The 1-D Matern-3/2 workload at n = 2^20: projected, log det within 1e-10 and
  the quadratic form within 1e-8 of the Kalman oracle.
* The smallest trees (a single leaf, one, two and three levels with uneven
  leaves): both forms against each other and the dense oracle.
"""
import numpy as np
import pytest

import oracle
import paper_1403_6015_amd as H
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _dev_call(p, opts, presorted=False):
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
    work = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    out = torch.zeros(8, dtype=torch.float64, device=dev)
    z = torch.zeros(p.n, dtype=torch.float64, device=dev)
    H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, work,
                    plan.workspace_bytes, None, out, z)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:3].copy(), z.cpu().numpy().copy(), plan.info()


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


CASES = [
    ("se1d", lambda: wl.random_problem(4096, 1, wl.K_SE, 701, ell=0.02, sigma2=0.02, leaf=64,
                                       tol=1e-12)),
    ("matern1d", lambda: wl.random_problem(6000, 1, wl.K_MATERN32, 702, ell=0.1, sigma2=0.05,
                                           leaf=64, tol=1e-12)),
    ("exp1d", lambda: wl.random_problem(3000, 1, wl.K_EXP, 703, ell=0.2, sigma2=0.05, leaf=64,
                                        tol=1e-12)),
    ("imq1d", lambda: wl.random_problem(2500, 1, wl.K_IMQ, 704, ell=0.05, sigma2=0.05, leaf=64,
                                        tol=1e-12)),
    ("se2d", lambda: wl.random_problem(3000, 2, wl.K_SE, 705, ell=1.0, sigma2=0.05, leaf=128,
                                       tol=1e-10)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [H.FP64, H.MIXED], ids=["fp64", "mixed"])
def test_projected_equals_level_by_level(name, make, precision):
    p = make()
    announce("projected vs level-by-level %s n=%d dim=%d precision=%d" % (name, p.n, p.dim,
                                                                           precision))
    kw = dict(max_rank=64, precision=precision, mixed_unchecked=1)
    o0, z0, i0 = _dev_call(p, H.Opts(level_form=0, **kw))
    o1, z1, i1 = _dev_call(p, H.Opts(level_form=1, **kw))
    print("  ranks %s projected %d/%d; logdet %.3e quad %.3e z %.3e" % (
        i0["rank_max"], i0["projected"], i1["projected"], _rel(o0[1], o1[1]),
        _rel(o0[2], o1[2]), np.linalg.norm(z0 - z1) / np.linalg.norm(z1)), flush=True)
    assert i0["projected"] == 1 and i1["projected"] == 0
    assert i0["rank_max"] == i1["rank_max"]
    # the mixed forms round their FP32 panels at different points
    assert _rel(o0[1], o1[1]) <= (1e-12 if precision == H.FP64 else 1e-8)
    assert _rel(o0[2], o1[2]) <= (1e-10 if precision == H.FP64 else 1e-6)
    # an unrefined FP32-panel solve is accurate to about 6e-8 times the
    # conditioning (||K|| / sigma^2 up to ~1e3 here), differently in each form
    assert np.linalg.norm(z0 - z1) <= (1e-9 if precision == H.FP64 else 1e-4) * np.linalg.norm(z1)
    ref = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    bar = 1e-10 if precision == H.FP64 else 1e-8
    assert _rel(o0[1], ref["logdet"]) <= bar


def test_wide_ranks_take_the_level_by_level_form():
    p = wl.random_problem(4096, 2, wl.K_SE, 706, ell=0.1, sigma2=0.01, leaf=128, tol=1e-10)
    announce("projected form limits: 2-D SE n=%d" % p.n)
    o0, z0, i0 = _dev_call(p, H.Opts(max_rank=64))
    o1, z1, i1 = _dev_call(p, H.Opts(max_rank=64, level_form=1))
    print("  ranks %s projected %d" % (i0["rank_max"], i0["projected"]), flush=True)
    assert max(i0["rank_max"]) > 32
    assert i0["projected"] == 0
    assert np.array_equal(o0, o1) and np.array_equal(z0, z1)


def test_batched_items_against_kalman():
    import torch
    n, m = 16384, 6
    x, y, th = wl.batched_theta(m=m, n=n)
    announce("projected batched n=%d m=%d" % (n, m))
    opts = H.Opts(max_rank=16, presorted=1)
    plan = H.Plan(n, 1, 128, opts)
    nb = plan.batch_workspace_bytes(m)
    d_x = torch.from_numpy(np.ascontiguousarray(x.reshape(1, -1))).cuda()
    d_y = torch.from_numpy(y).cuda()
    d_p = torch.from_numpy(np.ascontiguousarray(th)).cuda()
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    out = torch.full((m, 3), np.nan, dtype=torch.float64, device="cuda")
    H.gp_loglik_batch_dev(plan, d_x, H.K_MATERN32, d_p, m, d_y, 0, 1e-10, work, nb, None, out,
                          False)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    for i in range(m):
        a, ell, s2 = th[i]
        kf = oracle.kalman_matern32(x[:, 0], y, (a, ell), s2, want_alpha=False)
        assert abs(res[i, 1] - kf["logdet"]) <= 1e-10 * max(abs(kf["logdet"]), 1.0), i
        assert _rel(res[i, 2], kf["quad"]) <= 1e-8, i


def test_full_size_matern_projected():
    p = wl.matern1d(1 << 20)
    announce("projected 1-D Matern n=2^20")
    o, z, info = _dev_call(p, H.Opts(max_rank=64, presorted=1), presorted=True)
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, want_alpha=True)
    print("  projected %d; logdet rel %.2e quad rel %.2e z rel %.2e" % (
        info["projected"], _rel(o[1], kf["logdet"]), _rel(o[2], kf["quad"]),
        np.linalg.norm(z - kf["alpha"]) / np.linalg.norm(kf["alpha"])), flush=True)
    assert info["projected"] == 1
    assert _rel(o[1], kf["logdet"]) <= 1e-10
    assert _rel(o[2], kf["quad"]) <= 1e-8
    assert np.linalg.norm(z - kf["alpha"]) <= 1e-6 * np.linalg.norm(kf["alpha"])


def test_option_is_validated():
    with pytest.raises(H.HodlrError) as ei:
        H.Plan(4096, 1, 64, H.Opts(level_form=2))
    assert ei.value.name == "EINVAL"


@pytest.mark.parametrize("n", [64, 65, 130, 300])
def test_smallest_trees(n):
    """A single leaf (no level: the level-by-level form), one level (the root
    only) and two or three levels with uneven leaves: both forms against each
    other and the dense oracle."""
    p = wl.random_problem(n, 1, wl.K_MATERN32, 707 + n, ell=0.1, sigma2=0.05, leaf=64, tol=1e-12)
    announce("projected form, smallest trees: n=%d leaf=64" % n)
    o0, z0, i0 = _dev_call(p, H.Opts(max_rank=64))
    o1, z1, i1 = _dev_call(p, H.Opts(max_rank=64, level_form=1))
    print("  levels %d projected %d" % (i0["levels"], i0["projected"]), flush=True)
    assert i0["projected"] == (1 if i0["levels"] >= 1 else 0)
    assert _rel(o0[1], o1[1]) <= 1e-12 and _rel(o0[2], o1[2]) <= 1e-10
    assert np.linalg.norm(z0 - z1) <= 1e-10 * np.linalg.norm(z1)
    ref = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    assert _rel(o0[1], ref["logdet"]) <= 1e-10
    assert _rel(o0[2], ref["quad"]) <= 1e-9
