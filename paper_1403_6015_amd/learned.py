"""Surrogate-screened posterior sampling over GP hyperparameters.

Host orchestration of the library's device entry points for the paper's
outer loop (§1: the likelihood of Eq. (1) evaluated many times while
inferring theta).  Every likelihood, network pass, training step and sampler
decision runs in the library's kernels; this module only chooses inputs
(design points, random numbers) and reads results:

1. ``laplace``: a local quadratic model of l(log theta) from batched exact
   likelihoods on a cloud of points, iterated to the mode; -H^{-1} gives the
   scale of the posterior.
2. ``training_set``: exact likelihoods at design points drawn around the mode
   on two scales (the bulk and the tails the walkers start from).
3. ``train``: minibatch Adam on the device network.
4. ``sample``: plain or delayed-acceptance Metropolis with W walkers.
5. ``ess``: effective sample size by Sokal's automatic windowing.
"""
from __future__ import annotations

import time

import numpy as np

from . import (K_MATERN32, MLP_NPARAM, MlpNorm, Opts, Plan, SamplerCfg, gp_loglik_batch_dev,
               gp_sample_dev, mlp_cast_dev, mlp_fit_dev, mlp_forward_dev, mlp_workspace_size,
               sampler_workspace_size)


class ExactGP:
    """Shared points and observations on the device plus a plan, for batched
    exact log-likelihoods at many log-hyperparameters."""

    def __init__(self, x, y, kernel=K_MATERN32, leaf=128, tol=1e-10, max_rank=16, chunk=256):
        import torch
        self.torch = torch
        x = np.asarray(x, dtype=np.float64).reshape(len(y), -1)
        self.n, self.dim = x.shape
        self.kernel, self.tol, self.chunk = kernel, tol, chunk
        self.plan = Plan(self.n, self.dim, leaf, Opts(max_rank=max_rank))
        self.d_x = torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
        self.d_y = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float64)).cuda()
        self.wbytes = self.plan.batch_workspace_bytes(chunk)
        self.work = torch.empty(self.wbytes, dtype=torch.uint8, device="cuda")
        self.stream = torch.cuda.Stream()
        self.evals = 0

    def loglik(self, logtheta):
        """Exact log-likelihoods at rows of log theta (m x 3), chunked."""
        torch = self.torch
        lt = np.atleast_2d(np.asarray(logtheta, dtype=np.float64))
        out = np.empty(len(lt))
        with torch.cuda.stream(self.stream):
            for s in range(0, len(lt), self.chunk):
                part = lt[s:s + self.chunk]
                m = len(part)
                d_p = torch.from_numpy(np.exp(part)).cuda()
                d_o = torch.empty((m, 3), dtype=torch.float64, device="cuda")
                gp_loglik_batch_dev(self.plan, self.d_x, self.kernel, d_p, m, self.d_y, 0,
                                    self.tol, self.work, self.wbytes, self.stream, d_o, False)
                self.stream.synchronize()
                out[s:s + m] = d_o[:, 0].cpu().numpy()
        self.evals += len(lt)
        return out


def _quad_features(d):
    """[1, d_i, d_i d_j (i <= j)] for a quadratic fit in 3 variables."""
    cols = [np.ones(len(d))] + [d[:, i] for i in range(3)]
    for i in range(3):
        for j in range(i, 3):
            cols.append(d[:, i] * d[:, j])
    return np.stack(cols, axis=1)


def laplace(gp: ExactGP, center, scale, rounds=4, npts=96, seed=0):
    """Mode and covariance of exp(l) near ``center`` (log theta): each round
    fits l by least squares to a quadratic on a Gaussian cloud around the
    current centre, takes the Newton step (bounded by the cloud size) and
    shrinks the cloud to the implied posterior scale."""
    rng = np.random.default_rng(seed)
    c = np.asarray(center, dtype=np.float64).copy()
    s = np.full(3, float(scale)) if np.isscalar(scale) else np.asarray(scale, dtype=np.float64)
    cov = np.diag(s * s)
    for _ in range(rounds):
        d = rng.standard_normal((npts, 3)) * s
        ll = gp.loglik(c + d)
        ok = np.isfinite(ll)
        A = _quad_features(d[ok])
        coef, *_ = np.linalg.lstsq(A, ll[ok], rcond=None)
        g = coef[1:4]
        Hm = np.zeros((3, 3))
        k = 4
        for i in range(3):
            for j in range(i, 3):
                if i == j:
                    Hm[i, i] = 2 * coef[k]
                else:
                    Hm[i, j] = Hm[j, i] = coef[k]
                k += 1
        w, V = np.linalg.eigh(-Hm)
        w = np.maximum(w, 1e-12)
        cov = (V / w) @ V.T
        step = cov @ g
        lim = 2.0 * s
        step = np.clip(step, -lim, lim)
        c = c + step
        s = np.minimum(s, 3.0 * np.sqrt(np.diag(cov)))
    return c, cov


def training_set(gp: ExactGP, mode, cov, n=20000, wide=4.0, narrow=2.0, frac_wide=0.3, seed=1):
    """Design points log theta ~ N(mode, k^2 cov) with k = narrow or wide, and
    their exact log-likelihoods (non-finite values dropped)."""
    rng = np.random.default_rng(seed)
    Lc = np.linalg.cholesky(cov)
    nw = int(frac_wide * n)
    k = np.concatenate([np.full(nw, wide), np.full(n - nw, narrow)])
    X = mode + (rng.standard_normal((n, 3)) @ Lc.T) * k[:, None]
    T = gp.loglik(X)
    ok = np.isfinite(T)
    return X[ok], T[ok]


class Surrogate:
    """Device network: FP32 master, BF16 copy, Adam moments, normalization."""

    def __init__(self, seed=0):
        import torch
        self.torch = torch
        rng = np.random.default_rng(seed)
        parts = []
        for fan_in, size, bias in ((3, 384, False), (0, 128, True), (128, 16384, False),
                                   (0, 128, True), (128, 128, False), (0, 1, True)):
            if bias:
                parts.append(np.zeros(size))
            else:
                lim = 1.0 / np.sqrt(fan_in)
                parts.append(rng.uniform(-lim, lim, size=size))
        p = np.concatenate(parts).astype(np.float32)
        assert p.size == MLP_NPARAM
        self.master = torch.from_numpy(p).cuda()
        self.wb = torch.empty(MLP_NPARAM, dtype=torch.int16, device="cuda")
        self.m = torch.zeros(MLP_NPARAM, dtype=torch.float32, device="cuda")
        self.v = torch.zeros_like(self.m)
        mlp_cast_dev(self.master, self.wb)
        self.norm = MlpNorm()
        self.step = 1

    def fit(self, X, T, epochs=150, batch=256, lr=2e-3, seed=2):
        """Sets the normalization from the data and trains; returns the
        per-minibatch losses."""
        torch = self.torch
        X = np.asarray(X, dtype=np.float64)
        T = np.asarray(T, dtype=np.float64)
        mu, sd = X.mean(axis=0), X.std(axis=0)
        self.norm = MlpNorm(mu, sd, float(T.mean()), float(T.std()))
        N = len(T)
        g = torch.Generator().manual_seed(seed)
        perm = torch.cat([torch.randperm(N, generator=g) for _ in range(epochs)])
        perm = perm.to(torch.int32).cuda()
        nb = mlp_workspace_size(batch)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        per = (N + batch - 1) // batch
        hist = torch.empty(epochs * per, dtype=torch.float32, device="cuda")
        d_x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
        d_t = torch.from_numpy(np.ascontiguousarray(T)).cuda()
        mlp_fit_dev(self.master, self.wb, self.m, self.v, self.step, lr, self.norm, d_x, d_t, N,
                    perm, epochs, batch, work, nb, hist)
        torch.cuda.synchronize()
        self.step += epochs * per
        return hist.cpu().numpy()

    def predict(self, X):
        torch = self.torch
        X = np.ascontiguousarray(np.atleast_2d(X), dtype=np.float64)
        out = torch.empty(len(X), dtype=torch.float64, device="cuda")
        mlp_forward_dev(self.wb, self.norm, torch.from_numpy(X).cuda(), len(X), out)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def sample(gp: ExactGP, start, chol, lo, hi, steps, surrogate: Surrogate | None = None,
           seed=3, block=50):
    """Runs ``steps`` Metropolis steps of W = len(start) walkers in blocks of
    ``block`` steps (random numbers drawn per block on the device).  Returns
    (chain [steps, W, 3], tallies, seconds)."""
    torch = gp.torch
    start = np.ascontiguousarray(start, dtype=np.float64)
    W = len(start)
    nb = sampler_workspace_size(gp.plan, W)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    d_th = torch.from_numpy(start.copy()).cuda()
    d_lp = torch.empty(W, dtype=torch.float64, device="cuda")
    d_sur = torch.empty(W, dtype=torch.float64, device="cuda")
    chain = torch.empty((steps, W, 3), dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(seed)
    tallies = {"proposals": 0, "survivors": 0, "exact_evals": 0, "accepted": 0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    with torch.cuda.stream(gp.stream):
        while done < steps:
            k = min(block, steps - done)
            eps = torch.randn((k, W, 3), dtype=torch.float64, device="cuda", generator=gen)
            u1 = torch.rand((k, W), dtype=torch.float64, device="cuda", generator=gen)
            u2 = torch.rand((k, W), dtype=torch.float64, device="cuda", generator=gen)
            # uniforms in (0, 1): torch.rand may return 0, whose log is -inf (always accept)
            u1.clamp_(min=1e-300)
            u2.clamp_(min=1e-300)
            cfg = SamplerCfg(W, k, lo, hi, chol, init_state=1 if done == 0 else 0)
            t = gp_sample_dev(gp.plan, gp.d_x, gp.kernel, gp.d_y, gp.tol,
                              surrogate.wb if surrogate is not None else None,
                              surrogate.norm if surrogate is not None else None, cfg, d_th, d_lp,
                              d_sur, eps, u1, u2, work, nb, gp.stream, chain[done:done + k])
            for key in tallies:
                tallies[key] += t[key]
            done += k
        gp.stream.synchronize()
    secs = time.perf_counter() - t0
    gp.evals += tallies["exact_evals"]
    return chain.cpu().numpy(), tallies, secs


def bulk_rmse(pred, target, ref_loglik, window=15.0):
    """RMS error over the points whose exact log-likelihood lies within
    ``window`` nats of ref_loglik (the region the walkers occupy)."""
    pred, target = np.asarray(pred), np.asarray(target)
    b = target > ref_loglik - window
    return float(np.sqrt(np.mean((pred[b] - target[b]) ** 2))), int(b.sum())


def ess(x):
    """Effective sample size of one scalar chain: N / tau with the
    integrated autocorrelation time tau = 1 + 2 sum_{k<=M} rho_k, M the
    smallest lag with M >= 5 tau(M) (Sokal's automatic window)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    x = x - x.mean()
    v = float(np.dot(x, x))
    if v == 0.0 or n < 4:
        return float(n)
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(x, m)
    rho = np.fft.irfft(f * np.conj(f), m)[:n] / v
    tau = 1.0
    for lag in range(1, n):
        tau += 2.0 * rho[lag]
        if lag >= 5.0 * tau:
            break
    return float(n / max(tau, 1.0 / n))


def chain_ess(chain, burn=0):
    """Sum over walkers of the smallest per-coordinate ESS after ``burn``."""
    c = chain[burn:]
    tot = 0.0
    for w in range(c.shape[1]):
        tot += min(ess(c[:, w, k]) for k in range(c.shape[2]))
    return tot
