"""Leaves above 128 points and ranks above 64 (the 2-D configuration's leaf
256 and the caps it needs) against the FP64 dense oracle: the large-leaf
kernel (first 128 rows and the Schur complement in LDS, the off-diagonal
half through HBM), the level stage's wide path (MFMA products over rank
groups, coupling matrices in HBM), the stored-factor solve of large leaves,
and the device and batched entry points on such plans.

Bars as for the FP64 form elsewhere: log det within 1e-10 of the oracle
(relative), every solve at a 1e-10 relative residual (FP64 factors refine
against the exact product where a single application of the factor cannot
reach it: its residual is about tol ||K|| / sigma^2)."""
import math

import numpy as np
import pytest

import oracle
import paper_1403_6015_amd as H
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _check(p, leaf, opts, ld_tol=1e-10, res_tol=1e-10):
    announce("%s n=%d dim=%d leaf=%d tol=%g cap=%d" % (p.name, p.n, p.dim, leaf, p.tol,
                                                      opts.max_rank))
    ref = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    f = H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, leaf, p.tol, opts)
    ld = f.logdet()
    z = f.solve(p.y)
    info = f.info()
    f.free()
    C = oracle.dense_matrix(p.x, p.kernel, p.theta, p.sigma2)
    res = float(np.linalg.norm(p.y - C @ z) / np.linalg.norm(p.y))
    rel = abs(ld - ref["logdet"]) / max(abs(ref["logdet"]), 1.0)
    print("  leaf_max %d levels %d rank_max %s capped %d: logdet rel %.2e residual %.2e" % (
        info["leaf_max"], info["levels"], info["rank_max"], info["capped_blocks"], rel, res),
        flush=True)
    assert rel <= ld_tol, (rel, info)
    assert res <= res_tol, (res, info)
    ll, ld2, q = H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, leaf, p.tol, opts)
    assert abs(ld2 - ref["logdet"]) <= ld_tol * max(abs(ref["logdet"]), 1.0)
    assert abs(ll - ref["loglik"]) <= 1e-9 * max(abs(ref["loglik"]), 1.0)
    return info


@pytest.mark.parametrize("n,leaf", [(2048, 256), (3000, 200), (2100, 150), (4100, 129)])
def test_large_leaves_1d(n, leaf):
    """1-D SE with leaves of 129..256 points (including trees whose leaves
    straddle 128): the large-leaf factor and its stored-factor solve."""
    p = wl.random_problem(n, 1, wl.K_SE, seed=n + leaf, ell=0.1, sigma2=0.02, leaf=leaf,
                          tol=1e-12, lo=-1, hi=1)
    info = _check(p, leaf, H.Opts(max_rank=64))
    assert info["leaf_max"] == math.ceil(n / 2 ** info["levels"])
    assert info["leaf_max"] > 128


def test_large_leaves_matern_against_kalman():
    """Matern-3/2 at n = 2^16, leaf 256: log det, quadratic form and
    log-likelihood against the exact state-space recursion."""
    p = wl.matern1d(1 << 16)
    announce("matern n=%d leaf=256" % p.n)
    ll, ld, q = H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, 256, p.tol)
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, want_alpha=False)
    print("  logdet rel %.2e quad rel %.2e" % (abs(ld - kf["logdet"]) / abs(kf["logdet"]),
                                               abs(q - kf["quad"]) / abs(kf["quad"])))
    assert abs(ld - kf["logdet"]) <= 1e-12 * abs(kf["logdet"])
    assert abs(q - kf["quad"]) <= 1e-11 * abs(kf["quad"])


def test_wide_ranks_with_small_leaves():
    """2-D SE (l = 0.05, sigma^2 = 1e-2) on the unit square, n = 4096, leaf
    64, cap 512: the wide level path (ranks above 64 on most levels) with the
    LDS leaf kernel."""
    p = wl.se2d(4096, side=1.0)
    info = _check(p, 64, H.Opts(max_rank=512, refine=1))
    assert max(info["rank_max"]) > 64 and info["capped_blocks"] == 0


@pytest.mark.parametrize("n", [2048, 4096])
def test_2d_se_unit_square_leaf256_uncapped(n):
    """The 2-D configuration's kernel on the unit square at leaf 256 with the
    cap raised to 512 (no block capped): ranks far above 64 at every level."""
    p = wl.se2d(n, side=1.0)
    info = _check(p, 256, H.Opts(max_rank=512, refine=1))
    assert max(info["rank_max"]) > 128 and info["capped_blocks"] == 0


def test_2d_se_node_inverse_in_lds():
    """2-D SE on the square of side 1/4 (the density-matched n = 2^18 domain)
    with n = 8192, leaf 256, cap 128: the widest levels have ranks between 65
    and 128, whose node matrices are inverted in LDS (Gauss-Jordan), in the
    factorization and in the later solves."""
    p = wl.se2d(8192, side=0.25)
    info = _check(p, 256, H.Opts(max_rank=128, refine=1))
    assert 64 < max(info["rank_max"]) <= 128 and info["capped_blocks"] == 0


def test_2d_se_density_matched_leaf256():
    """n = 2^14 points on the sub-square of the n = 2^22 unit square's
    density (side 1/16), leaf 256, cap 128."""
    p = wl.se2d(1 << 14)
    info = _check(p, 256, H.Opts(max_rank=128, refine=1))
    assert info["leaf_max"] == 256


def test_wide_device_and_batched_entry_points():
    """gp_loglik_dev and gp_loglik_batch_dev on a leaf-256, cap-512 plan
    (tree-ordered points): the same log-likelihood as the host entry point
    and as each other."""
    import torch
    p = wl.se2d(2048, side=1.0)
    announce("wide plan device entry points n=%d" % p.n)
    perm = H.hodlr_order(p.x, 256)
    xo = p.x[perm]
    yo = p.y[perm]
    opts = H.Opts(max_rank=512, presorted=1)
    ll, ld, q = H.gp_loglik(xo, yo, p.kernel, p.theta, p.sigma2, 256, p.tol, opts)
    ref = oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    assert abs(ld - ref["logdet"]) <= 1e-10 * abs(ref["logdet"])
    plan = H.Plan(p.n, 2, 256, opts)
    dev = torch.device("cuda:0")
    d_x = torch.from_numpy(np.ascontiguousarray(xo.T)).to(dev)
    d_y = torch.from_numpy(yo).to(dev)
    work = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    out = torch.zeros(8, dtype=torch.float64, device=dev)
    H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, work,
                    plan.workspace_bytes, None, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert abs(o[1] - ld) <= 1e-12 * abs(ld)
    assert abs(o[0] - ll) <= 1e-12 * abs(ll)
    m = 3
    th = np.array([[1.0, 0.05, 1e-2], [0.8, 0.07, 2e-2], [1.2, 0.04, 1e-2]])
    nb = plan.batch_workspace_bytes(m)
    wb = torch.empty(nb, dtype=torch.uint8, device=dev)
    ob = torch.full((m, 3), np.nan, dtype=torch.float64, device=dev)
    H.gp_loglik_batch_dev(plan, d_x, p.kernel, torch.from_numpy(th).to(dev), m, d_y, 0, p.tol,
                          wb, nb, None, ob, False)
    torch.cuda.synchronize()
    res = ob.cpu().numpy()
    for i in range(m):
        r = oracle.gp_dense(p.x, p.y, p.kernel, tuple(th[i, :2]), th[i, 2])
        rel = abs(res[i, 1] - r["logdet"]) / abs(r["logdet"])
        print("  item %d logdet rel %.2e" % (i, rel), flush=True)
        assert rel <= 1e-10, i
