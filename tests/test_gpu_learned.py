"""GPU parity of the surrogate network and the sampler kernels against the
FP64 oracles: the BF16 weight copy bit for bit, the forward pass within a
bound derived from BF16 rounding of the hidden activations, the gradient element
by element, Adam's first step, and the sampler's stage kernels decision
for decision on oracle-supplied likelihood values; then the sampler driver's
invariants on a small GP."""
import numpy as np
import pytest

import oracle
import paper_1403_6015_amd as H
import workloads as wl
from oracle import mcmc_ref as mc
from oracle import mlp_ref as mr

pytestmark = pytest.mark.gpu

NORM = {"mu_in": np.array([0.1, -0.3, 0.2]), "sd_in": np.array([0.5, 1.5, 0.8]),
        "mu_out": 3.0, "sd_out": 2.5}
U8 = 2.0 ** -8    # BF16 unit roundoff


def announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _norm():
    return H.MlpNorm(NORM["mu_in"], NORM["sd_in"], NORM["mu_out"], NORM["sd_out"])


def _params(seed):
    rng = np.random.default_rng(seed)
    p = mr.init_params(seed) + 0.05 * rng.standard_normal(mr.NPARAM)
    return p.astype(np.float32)   # the FP32 master copy


def _device_net(p32):
    import torch
    dev = torch.device("cuda:0")
    master = torch.from_numpy(p32.copy()).to(dev)
    wb = torch.empty(mr.NPARAM, dtype=torch.int16, device=dev)
    H.mlp_cast_dev(master, wb)
    torch.cuda.synchronize()
    return master, wb


def _bf16_from_bits(bits):
    return (bits.astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def test_bf16_copy_is_round_to_nearest_even():
    announce("mlp cast")
    p32 = _params(1)
    _, wb = _device_net(p32)
    got = _bf16_from_bits(wb.cpu().numpy().view(np.uint16))
    assert np.array_equal(got, mr.bf16_round(p32.astype(np.float64)))


@pytest.mark.parametrize("batch", [1, 31, 100, 257])
def test_forward_matches_oracle(batch):
    import torch
    announce("mlp forward batch=%d" % batch)
    p32 = _params(2)
    _, wb = _device_net(p32)
    pb = mr.bf16_round(p32.astype(np.float64))
    X = np.random.default_rng(batch).normal(size=(batch, 3))
    d_x = torch.from_numpy(X).cuda()
    d_o = torch.full((batch,), np.nan, dtype=torch.float64, device="cuda")
    H.mlp_forward_dev(wb, _norm(), d_x, batch, d_o)
    torch.cuda.synchronize()
    got = d_o.cpu().numpy()
    ref, c = mr.forward(pb, X, NORM)
    P = mr.unpack(pb)
    # the device rounds h1 to BF16 before the 128-wide product: per sample
    # |d o| <= sum_o |W3_o| sum_i |W2_oi| |h1_i| u8, plus FP32 arithmetic
    bound = U8 * (np.abs(c["H1"]) @ np.abs(P["W2"]).T) @ np.abs(P["W3"])
    bound += 1e-5 * (1.0 + np.abs(P["W3"]).sum())
    err = np.abs(got - ref) / NORM["sd_out"]
    assert np.all(err <= bound), (err.max(), bound.min())


def _grad_terms(p, X, T):
    """Per gradient entry: the sum of |terms| of the sums that form it, and the
    largest single |term| (the oracle's chain rule with absolute values)."""
    P = mr.unpack(p)
    _, c = mr.forward(p, X, NORM)
    B = X.shape[0]
    go = 2.0 * (c["O"] - (T - NORM["mu_out"]) / NORM["sd_out"]) / B
    ad = np.abs(go[:, None] * P["W3"][None, :] * (1 - c["H2"] ** 2))
    mz1 = (ad @ np.abs(P["W2"])) * (1 - c["H1"] ** 2)
    aU, aH1, aH2, ag = np.abs(c["U"]), np.abs(c["H1"]), np.abs(c["H2"]), np.abs(go)
    mag = np.concatenate([(mz1.T @ aU).ravel(), mz1.sum(0), (ad.T @ aH1).ravel(), ad.sum(0),
                          aH2.T @ ag, [ag.sum()]])
    big = np.concatenate([np.max(mz1[:, :, None] * aU[:, None, :], axis=0).ravel(), mz1.max(0),
                          np.max(ad[:, :, None] * aH1[:, None, :], axis=0).ravel(), ad.max(0),
                          (aH2 * ag[:, None]).max(0), [ag.max()]])
    return mag, big


def test_gradient_matches_oracle_element_by_element():
    """Every one of the 17153 gradient entries against the oracle's gradient
    with the same BF16 operands (h1 and dz2 rounded where they enter the two
    128-wide products).  What remains is FP32 arithmetic (accumulation order,
    tanhf) and the rare BF16 rounding decision that FP32 and FP64 values take
    differently: per entry 1e-5 of its summed term magnitudes plus 4 unit
    roundoffs of its largest single term."""
    import torch
    B = 200
    announce("mlp gradient batch=%d" % B)
    p32 = _params(3)
    _, wb = _device_net(p32)
    pb = mr.bf16_round(p32.astype(np.float64))
    rng = np.random.default_rng(30)
    X = rng.normal(size=(B, 3))
    T = rng.normal(3.0, 4.0, size=B)
    loss_ref, g_ref = mr.loss_and_grad(pb, X, T, NORM, bf16_products=True)
    mag, big = _grad_terms(pb, X, T)
    nb = H.mlp_workspace_size(B)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    grad = torch.empty(mr.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    H.mlp_grad_dev(wb, _norm(), torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), B, work,
                   nb, grad, loss)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - loss_ref) <= 1e-4 * loss_ref
    bound = 1e-5 * mag + 4 * U8 * big + 1e-9
    err = np.abs(g - g_ref)
    worst = int(np.argmax(err / bound))
    print("mlp gradient: worst entry %d err %.3e bound %.3e; median bound / |g| %.2e" % (
        worst, err[worst], bound[worst], np.median(bound / (np.abs(g_ref) + 1e-12))))
    assert np.all(err <= bound), (worst, err[worst], bound[worst])


def test_adam_first_step_matches_oracle():
    import torch
    B = 64
    announce("mlp adam step")
    p32 = _params(4)
    master, wb = _device_net(p32)
    pb = mr.bf16_round(p32.astype(np.float64))
    rng = np.random.default_rng(40)
    X = rng.normal(size=(B, 3))
    T = rng.normal(3.0, 4.0, size=B)
    _, g_ref = mr.loss_and_grad(pb, X, T, NORM)
    m = torch.zeros(mr.NPARAM, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    nb = H.mlp_workspace_size(B)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    lr = 1e-3
    H.mlp_train_step_dev(master, wb, m, v, 1, lr, _norm(), torch.from_numpy(X).cuda(),
                         torch.from_numpy(T).cuda(), B, work, nb)
    torch.cuda.synchronize()
    step = master.cpu().numpy().astype(np.float64) - p32.astype(np.float64)
    p1, _, _ = mr.adam_step(p32.astype(np.float64), 0.0, 0.0, g_ref, 1, lr)
    ref = p1 - p32
    # at t = 1 the step is lr g / (|g| + eps): lr times the gradient's sign
    # wherever |g| is well above the device's relative error of g
    big = np.abs(g_ref) > 5e-2 * np.abs(g_ref).max()
    assert np.all(np.sign(step[big]) == np.sign(ref[big]))
    assert np.allclose(step[big], ref[big], rtol=1e-3, atol=lr * 1e-6)
    wb_host = _bf16_from_bits(wb.cpu().numpy().view(np.uint16))
    assert np.array_equal(wb_host, mr.bf16_round(master.cpu().numpy().astype(np.float64)))


def test_fit_learns_a_smooth_function():
    import torch
    announce("mlp fit quadratic")
    rng = np.random.default_rng(50)
    N = 4096
    X = rng.uniform(-1, 1, size=(N, 3))
    T = 5.0 - 3.0 * X[:, 0] ** 2 - 2.0 * (X[:, 1] - 0.3) ** 2 - X[:, 2] * X[:, 0]
    nm = H.MlpNorm((0, 0, 0), (0.6, 0.6, 0.6), float(T.mean()), float(T.std()))
    p32 = mr.init_params(7).astype(np.float32)
    master, wb = _device_net(p32)
    m = torch.zeros(mr.NPARAM, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    epochs, batch = 60, 256
    g = torch.Generator().manual_seed(51)
    perm = torch.cat([torch.randperm(N, generator=g) for _ in range(epochs)]).to(torch.int32).cuda()
    nb = H.mlp_workspace_size(batch)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    per = (N + batch - 1) // batch
    hist = torch.empty(epochs * per, dtype=torch.float32, device="cuda")
    H.mlp_fit_dev(master, wb, m, v, 1, 3e-3, nm, torch.from_numpy(X).cuda(),
                  torch.from_numpy(T).cuda(), N, perm, epochs, batch, work, nb, hist)
    torch.cuda.synchronize()
    h = hist.cpu().numpy()
    assert np.all(np.isfinite(h))
    assert h[-per:].mean() < 0.02 * h[:per].mean()
    # held-out error through the oracle forward with the trained BF16 weights
    Xt = rng.uniform(-1, 1, size=(500, 3))
    Tt = 5.0 - 3.0 * Xt[:, 0] ** 2 - 2.0 * (Xt[:, 1] - 0.3) ** 2 - Xt[:, 2] * Xt[:, 0]
    pb = _bf16_from_bits(wb.cpu().numpy().view(np.uint16))
    pred, _ = mr.forward(pb, Xt, nm.as_dict())
    assert np.sqrt(np.mean((pred - Tt) ** 2)) < 0.1 * Tt.std()


def test_sampler_stage_kernels_match_oracle_decisions():
    import torch
    announce("sampler stage kernels")
    rng = np.random.default_rng(60)
    W = 200
    lo, hi = np.array([-1.0, -2.0, -3.0]), np.array([1.0, 0.5, 0.0])
    th = rng.uniform(lo, hi, size=(W, 3))
    L = np.array([[0.3, 0, 0], [0.1, 0.2, 0], [-0.05, 0.02, 0.25]])
    eps = rng.standard_normal((W, 3))
    u1, u2 = rng.uniform(size=W), rng.uniform(size=W)
    lp = rng.normal(-100, 3, size=W)
    sur = lp + rng.normal(0, 0.5, size=W)
    prop = mc.propose(th, L, eps)
    sur_prop = rng.normal(-100, 3, size=W)
    lp_prop = sur_prop + rng.normal(0, 0.5, size=W)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()   # noqa: E731
    d_th, d_eps, d_prop = cu(th), cu(eps), torch.empty((W, 3), dtype=torch.float64, device="cuda")
    H.mh_propose_dev(W, d_th, L, d_eps, d_prop)
    torch.cuda.synchronize()
    assert np.allclose(d_prop.cpu().numpy(), prop, rtol=0, atol=1e-14)
    for delayed in (True, False):
        d_prop = cu(prop)   # the oracle's proposals drive both sides from here
        slot = torch.empty(W, dtype=torch.int32, device="cuda")
        count = torch.empty(1, dtype=torch.int32, device="cuda")
        params = torch.empty((W, 3), dtype=torch.float64, device="cuda")
        H.da_screen_dev(W, d_prop, lo, hi, cu(sur), cu(sur_prop) if delayed else None, cu(u1),
                        slot, count, params)
        torch.cuda.synchronize()
        surv = mc.da_stage1(sur, sur_prop, prop, u1, lo, hi) if delayed else mc.in_box(prop, lo, hi)
        c = int(surv.sum())
        assert count.item() == c
        sl = slot.cpu().numpy()
        assert np.array_equal(sl >= 0, surv)
        assert np.array_equal(sl[surv], np.arange(c))
        assert np.allclose(params.cpu().numpy()[:c], np.exp(prop[surv]), rtol=1e-15, atol=0)
        exact = np.zeros((W, 3))
        exact[:c, 0] = lp_prop[surv]
        d_th2, d_lp, d_sur = cu(th), cu(lp), cu(sur)
        acc = torch.empty(W, dtype=torch.int32, device="cuda")
        H.da_accept_dev(W, delayed, slot, cu(exact), cu(u2 if delayed else u1), d_prop,
                        cu(sur_prop), d_th2, d_lp, d_sur, acc)
        torch.cuda.synchronize()
        if delayed:
            t_ref, l_ref, s_ref, a_ref = mc.da_stage2(th, lp, sur, prop, lp_prop, sur_prop, surv, u2)
            assert np.array_equal(d_sur.cpu().numpy(), s_ref)
        else:
            t_ref, l_ref, a_ref = mc.mh_step(th, lp, prop, lp_prop, u1, lo, hi)
        assert np.array_equal(acc.cpu().numpy().astype(bool), a_ref)
        assert np.array_equal(d_th2.cpu().numpy(), t_ref)
        assert np.array_equal(d_lp.cpu().numpy(), l_ref)


@pytest.mark.parametrize("delayed", [False, True])
def test_sampler_driver_invariants_on_a_small_gp(delayed):
    import torch
    announce("sampler driver delayed=%s" % delayed)
    n, W, steps = 2048, 24, 12
    p = wl.matern1d(n)
    plan = H.Plan(n, 1, p.leaf, H.Opts(max_rank=16))
    d_x = torch.from_numpy(np.ascontiguousarray(p.x.T)).cuda()
    d_y = torch.from_numpy(p.y).cuda()
    t0 = np.log([p.theta[0], p.theta[1], p.sigma2])
    lo, hi = t0 - 1.0, t0 + 1.0
    rng = np.random.default_rng(70)
    th = t0 + 0.1 * rng.standard_normal((W, 3))
    L = 0.05 * np.eye(3)
    cfg = H.SamplerCfg(W, steps, lo, hi, L, init_state=1)
    p32 = _params(8)
    nm = H.MlpNorm(t0, (0.5, 0.5, 0.5), -3000.0, 50.0)
    _, wb = _device_net(p32)
    d_th = torch.from_numpy(th).cuda()
    d_lp = torch.empty(W, dtype=torch.float64, device="cuda")
    d_sur = torch.empty(W, dtype=torch.float64, device="cuda")
    eps = torch.from_numpy(rng.standard_normal((steps, W, 3))).cuda()
    u1 = torch.from_numpy(rng.uniform(size=(steps, W))).cuda()
    u2 = torch.from_numpy(rng.uniform(size=(steps, W))).cuda()
    nb = H.sampler_workspace_size(plan, W)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    chain = torch.empty((steps, W, 3), dtype=torch.float64, device="cuda")
    st = H.gp_sample_dev(plan, d_x, p.kernel, d_y, p.tol, wb if delayed else None,
                         nm if delayed else None, cfg, d_th, d_lp, d_sur, eps, u1, u2, work, nb,
                         None, chain)
    torch.cuda.synchronize()
    ch = chain.cpu().numpy()
    thf, lpf = d_th.cpu().numpy(), d_lp.cpu().numpy()
    assert np.array_equal(ch[-1], thf)
    assert np.all((ch >= lo) & (ch <= hi))
    assert st["proposals"] == steps * W
    assert st["exact_evals"] == W + st["survivors"]
    assert st["accepted"] <= st["survivors"]
    moved = np.any(ch[1:] != ch[:-1], axis=2).sum() + np.any(ch[0] != th, axis=1).sum()
    assert moved == st["accepted"]
    # the carried log-likelihood is the exact one at the carried point
    for i in range(0, W, 6):
        a, ell, s2 = np.exp(thf[i])
        kf = oracle.kalman_matern32(p.x[:, 0], p.y, (a, ell), s2, want_alpha=False)
        assert abs(lpf[i] - kf["loglik"]) <= 1e-9 * abs(kf["loglik"]), i
    if delayed:
        pb = _bf16_from_bits(wb.cpu().numpy().view(np.uint16))
        sref, _ = mr.forward(pb, thf, nm.as_dict())
        assert np.allclose(d_sur.cpu().numpy(), sref, rtol=0, atol=0.05 * 50.0)
