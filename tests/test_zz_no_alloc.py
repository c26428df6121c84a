"""The allocation-free training step against the workspace one: the same
state after two steps in a row (the second on a smaller batch), bit for bit,
and the batch limit rejected on the host."""
import numpy as np
import pytest

import paper_1403_6015_amd as H
from oracle import mlp_ref as mr

pytestmark = pytest.mark.gpu

NORM = (np.array([0.1, -0.3, 0.2]), np.array([0.5, 1.5, 0.8]), 3.0, 2.5)


def _state(torch, p32):
    dev = torch.device("cuda:0")
    master = torch.from_numpy(p32.copy()).to(dev)
    wb = torch.empty(mr.NPARAM, dtype=torch.int16, device=dev)
    H.mlp_cast_dev(master, wb)
    m = torch.zeros(mr.NPARAM, dtype=torch.float32, device=dev)
    v = torch.zeros_like(m)
    return master, wb, m, v


def test_noalloc_train_step_matches_workspace_step():
    import torch
    print("[gpu-case] mlp train step without allocation: batches 3000 then 45", flush=True)
    norm = H.MlpNorm(*NORM)
    rng = np.random.default_rng(77)
    p32 = (mr.init_params(7) + 0.05 * rng.standard_normal(mr.NPARAM)).astype(np.float32)
    ref = _state(torch, p32)
    got = _state(torch, p32)
    lr = 2e-3
    for step, B in ((1, 3000), (2, 45)):
        X = torch.from_numpy(rng.normal(size=(B, 3))).cuda()
        T = torch.from_numpy(rng.normal(3.0, 4.0, size=B)).cuda()
        nb = H.mlp_workspace_size(B)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        loss_ref = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        loss_got = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        H.mlp_train_step_dev(*ref, step, lr, norm, X, T, B, work, nb, d_loss=loss_ref)
        H.mlp_train_step_noalloc_dev(*got, step, lr, norm, X, T, B, d_loss=loss_got)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b), "step %d (batch %d) differs" % (step, B)
        assert torch.equal(loss_ref, loss_got) and bool(torch.isfinite(loss_got).all())
        print("step %d batch %d: state and loss identical (loss %.6f)"
              % (step, B, float(loss_got)), flush=True)


def test_noalloc_train_step_rejects_batches_beyond_its_limit():
    import torch
    norm = H.MlpNorm(*NORM)
    master, wb, m, v = _state(torch, mr.init_params(3).astype(np.float32))
    B = H.MLP_NOALLOC_MAX_BATCH + 1
    X = torch.zeros((B, 3), dtype=torch.float64, device="cuda")
    T = torch.zeros(B, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HodlrError) as e:
        H.mlp_train_step_noalloc_dev(master, wb, m, v, 1, 1e-3, norm, X, T, B)
    assert e.value.name == "EINVAL"
    with pytest.raises(H.HodlrError):
        H.mlp_train_step_noalloc_dev(master, wb, m, v, 1, 1e-3, norm, X, T, 0)
