"""GPU tests of the launch-shape autotuner: every tile shape gives the same
likelihood (the tiles only reorder sums), tuned plans match the Kalman
oracle, and the tuner's choice is the fastest of the times it reports and is
found again by the lookup."""
import numpy as np
import pytest

import oracle
import paper_1403_6015_amd as H
import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _dev_loglik(p, plan):
    import torch
    d_x = torch.from_numpy(np.ascontiguousarray(p.x.T)).cuda()
    d_y = torch.from_numpy(p.y.copy()).cuda()
    work = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, work,
                    plan.workspace_bytes, None, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:3]


@pytest.mark.parametrize("precision", [H.FP64, H.MIXED])
def test_tile_shapes_give_the_same_likelihood(precision):
    n = 1 << 16
    p = wl.matern1d(n)
    announce("tile shapes n=%d precision=%d" % (n, precision))
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, want_alpha=False)
    res = []
    for rows in (256, 512, 1024):
        for cols in (4, 8):
            for grp in (8, 64):
                t = H.Tune(128, rows, cols, grp)
                plan = H.Plan(n, 1, 128, H.Opts(max_rank=16, precision=precision), tune=t)
                res.append(_dev_loglik(p, plan))
    res = np.array(res)
    # FP64: reordered sums only; mixed: a reordered FP64 sum can move an FP32
    # store of W~ by one unit in the last place, which the coupling solves carry
    # on (measured 2e-11 relative across the six shapes)
    same = 1e-12 if precision == H.FP64 else 1e-9
    assert np.all(np.abs(res[:, 1] - res[0, 1]) <= same * abs(res[0, 1]))
    assert np.all(np.abs(res[:, 2] - res[0, 2]) <= (1e-12 if precision == H.FP64 else 1e-7)
                  * abs(res[0, 2]))
    tol = 1e-10 if precision == H.FP64 else 1e-8
    assert abs(res[0, 1] - kf["logdet"]) <= tol * abs(kf["logdet"])


def test_bad_tiles_are_rejected():
    with pytest.raises(H.HodlrError) as e:
        H.Plan(4096, 1, 64, None, tune=H.Tune(64, 300, 4))
    assert e.value.name == "EINVAL"
    with pytest.raises(H.HodlrError) as e:
        H.Plan(4096, 1, 64, None, tune=H.Tune(64, 512, 4, 16))
    assert e.value.name == "EINVAL"


def test_autotune_picks_its_fastest_candidate_and_caches_it():
    n = 1 << 17
    p = wl.matern1d(n)
    announce("autotune n=%d" % n)
    best, times = H.autotune(p.x, p.y, p.kernel, p.theta, p.sigma2, p.tol, H.Opts(max_rank=16),
                             leaf_cands=[64, 128], reps=2)
    assert len(times) == 2 + 12 and all(t > 0 for t in times)
    assert best.leaf in (64, 128)
    assert best.level_rows in (256, 512, 1024) and best.reduce_cols in (4, 8)
    assert min(times) == pytest.approx(min(times[:2] + times[2:]))
    # the winner is the fastest timed candidate
    shapes = [(64, 512, 4, 8), (128, 512, 4, 8)] + [(best.leaf, r, c, g) for r in (256, 512, 1024)
                                                    for c in (4, 8) for g in (8, 64)]
    assert shapes[int(np.argmin(times))] == (best.leaf, best.level_rows, best.reduce_cols,
                                             best.reduce_group)
    again = H.tune_lookup(n, 1, p.kernel, H.FP64)
    assert again.as_dict() == best.as_dict()
    plan = H.Plan(n, 1, best.leaf, H.Opts(max_rank=16), tune=best)
    o = _dev_loglik(p, plan)
    kf = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, want_alpha=False)
    assert abs(o[1] - kf["logdet"]) <= 1e-10 * abs(kf["logdet"])
    with pytest.raises(H.HodlrError):
        H.tune_lookup(3, 2, H.K_SE, H.MIXED)
