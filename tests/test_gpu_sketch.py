"""GPU parity of the randomized (sketch) compressor, HODLR_COMPRESS_SKETCH.

* 2-D squared exponential (the side-1/4 square, l = 0.1, sigma^2 = 1e-2),
  leaf 128, tol 1e-10, cap 64 (no block capped): the per-depth rank maxima and
  means equal those of the oracle's HODLR reference with the same compressor
  (same random signs; the SVD of the core is numpy's there, Jacobi here),
  the log det is within 1e-11 of that reference and within 1e-9 of the dense
  oracle, and the refined solve meets the 1e-10 residual bar.
* 1-D Matern-3/2 at the benchmark workload's density against the Kalman oracle.
* A capped case (the side-1/4 square with l = 0.05, cap 32: 15 blocks
  capped, still positive definite): the capped-block count and the rank
  maxima equal the reference's.
* The device entry point on a sketch plan equals the host one; the batched
  and uneven-size forms reject the compressor.
"""
import numpy as np
import pytest

import oracle
from oracle import hodlr_ref as hr
import paper_1403_6015_amd as H
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _ref_rank_stats(R):
    mx = [max(r) if r else 0 for r in R.ranks]
    mean = [float(np.mean(r)) if r else 0.0 for r in R.ranks]
    return mx, mean


def _sq(n, side, ell, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, side, (n, 2))
    y = rng.standard_normal(n)
    return x, y, (1.0, ell)


@pytest.mark.parametrize("n", [2048, 4096])
def test_2d_against_sketch_reference_and_dense(n):
    x, y, th = _sq(n, 0.25, 0.1, 500 + n)
    s2, tol, leaf = 1e-2, 1e-10, 128
    announce("sketch 2-D SE n=%d leaf=%d tol=%g" % (n, leaf, tol))
    opts = H.Opts(max_rank=64, compressor=H.COMPRESS_SKETCH, refine=1)
    f = H.hodlr_build(x, H.K_SE, th, s2, leaf, tol, opts)
    ld = f.logdet()
    z = f.solve(y)
    info = f.info()
    f.free()
    R = hr.HodlrRef(x, H.K_SE, th, s2, leaf, tol, max_rank=64, compress="sketch")
    mx, mean = _ref_rank_stats(R)
    L = info["levels"]
    print("  ranks gpu %s ref %s; capped %d/%d" % (info["rank_max"][:L], mx, info["capped_blocks"],
                                                     R.capped), flush=True)
    assert info["rank_max"][:L] == mx
    assert np.allclose(info["rank_mean"][:L], mean, rtol=0, atol=1e-12)
    assert info["capped_blocks"] == R.capped == 0
    ref = oracle.gp_dense(x, y, H.K_SE, th, s2)
    e_ref = abs(ld - R.logdet()) / abs(R.logdet())
    e_dense = abs(ld - ref["logdet"]) / abs(ref["logdet"])
    C = oracle.dense_matrix(x, H.K_SE, th, s2)
    res = np.linalg.norm(y - C @ z) / np.linalg.norm(y)
    print("  logdet vs sketch reference %.2e, vs dense %.2e; residual %.2e" % (e_ref, e_dense, res),
          flush=True)
    assert e_ref <= 1e-11
    assert e_dense <= 1e-9
    assert res <= 1e-10
    ll, ld2, q = H.gp_loglik(x, y, H.K_SE, th, s2, leaf, tol, opts)
    assert abs(ld2 - ld) <= 1e-13 * abs(ld)
    assert abs(ll - ref["loglik"]) <= 1e-9 * abs(ref["loglik"])


def test_1d_matern_against_kalman():
    p = wl.matern1d(1 << 14)
    announce("sketch 1-D Matern n=%d" % p.n)
    opts = H.Opts(max_rank=64, compressor=H.COMPRESS_SKETCH, presorted=1)
    ll, ld, q = H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, opts)
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, want_alpha=False)
    print("  logdet rel %.2e quad rel %.2e" % (abs(ld - kf["logdet"]) / abs(kf["logdet"]),
                                              abs(q - kf["quad"]) / abs(kf["quad"])), flush=True)
    assert abs(ld - kf["logdet"]) <= 1e-10 * abs(kf["logdet"])
    assert abs(q - kf["quad"]) <= 1e-8 * abs(kf["quad"])


def test_capped_case_counts_match_reference():
    x, y, th = _sq(4096, 0.25, 0.05, 77)
    announce("sketch capped 2-D n=4096 cap 32")
    opts = H.Opts(max_rank=32, compressor=H.COMPRESS_SKETCH)
    f = H.hodlr_build(x, H.K_SE, th, 1e-2, 128, 1e-10, opts)
    info = f.info()
    ld = f.logdet()
    f.free()
    R = hr.HodlrRef(x, H.K_SE, th, 1e-2, 128, 1e-10, max_rank=32, compress="sketch")
    mx, _ = _ref_rank_stats(R)
    L = info["levels"]
    print("  capped gpu %d ref %d; ranks %s" % (info["capped_blocks"], R.capped,
                                               info["rank_max"][:L]), flush=True)
    assert info["capped_blocks"] == R.capped > 0
    assert info["rank_max"][:L] == mx
    assert abs(ld - R.logdet()) <= 1e-10 * abs(R.logdet())


def test_device_entry_point_and_rejections():
    import torch
    x, y, th = _sq(2048, 0.25, 0.1, 31)
    announce("sketch plan device entry point n=2048")
    perm = H.hodlr_order(x, 128)
    xo, yo = x[perm], y[perm]
    opts = H.Opts(max_rank=64, compressor=H.COMPRESS_SKETCH, presorted=1)
    ll, ld, q = H.gp_loglik(xo, yo, H.K_SE, th, 1e-2, 128, 1e-10, opts)
    plan = H.Plan(2048, 2, 128, opts)
    dev = torch.device("cuda:0")
    d_x = torch.from_numpy(np.ascontiguousarray(xo.T)).to(dev)
    d_y = torch.from_numpy(yo).to(dev)
    work = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    out = torch.zeros(8, dtype=torch.float64, device=dev)
    H.gp_loglik_dev(plan, d_x, H.K_SE, th, 1e-2, d_y, 1e-10, work, plan.workspace_bytes, None, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert abs(o[1] - ld) <= 1e-13 * abs(ld)
    assert abs(o[0] - ll) <= 1e-12 * abs(ll)
    nb = plan.batch_workspace_bytes(2)
    wb = torch.empty(nb, dtype=torch.uint8, device=dev)
    params = torch.tensor([[1.0, 0.1, 1e-2], [1.0, 0.12, 1e-2]], dtype=torch.float64, device=dev)
    ob = torch.zeros((2, 3), dtype=torch.float64, device=dev)
    with pytest.raises(H.HodlrError) as ei:
        H.gp_loglik_batch_dev(plan, d_x, H.K_SE, params, 2, d_y, 0, 1e-10, wb, nb, None, ob, False)
    assert ei.value.name == "EINVAL"
    with pytest.raises(H.HodlrError) as ei:
        H.gp_loglik_ragged([x[:1000], x[:1500]], [y[:1000], y[:1500]], H.K_SE,
                           [[1.0, 0.1, 1e-2]] * 2, 128, 1e-10, opts)
    assert ei.value.name == "EINVAL"
