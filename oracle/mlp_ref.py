"""Surrogate network and its training step, written plainly in numpy (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper motivates fast likelihoods by the outer loop that needs many of them
(§1: hyperparameter inference, Eq. (1) and the posterior sampling that
follows it).  The learned surrogate is a small fully connected network that
maps log-hyperparameters to the log-likelihood:

    u   = (log theta - mu_in) / sd_in                       (3 inputs)
    h1  = tanh(W1 u + b1)                                   (128)
    h2  = tanh(W2 h1 + b2)                                  (128)
    o   = W3 . h2 + b3                                      (1)
    l~  = mu_out + sd_out * o

Parameters are one flat vector in the order W1 (128 x 3, row = unit),
b1 (128), W2 (128 x 128, row = output unit), b2 (128), W3 (128), b3 (1):
17153 numbers.  The loss of a batch of B pairs (log theta_s, l_s) is the mean
squared error in the standardized output, mean_s (o_s - (l_s - mu_out)/sd_out)^2.

Gradients are the chain rule written out layer by layer; the optimizer is
Adam as published by Kingma and Ba (2015), Algorithm 1, with bias-corrected
first and second moments.  Weights are never rounded here: a caller that
wants the oracle to see the network a BF16 device holds passes the rounded
weights.  ``loss_and_grad(..., bf16_products=True)`` also rounds the two
operands of each 128-wide product to BF16, the precision a BF16 matrix unit
takes them in; the default keeps every value FP64.
"""
from __future__ import annotations

import numpy as np

NIN, NH = 3, 128
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)),
         ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    """Flat vector -> dict of views in the order of ``SIZES``."""
    p = np.asarray(p, dtype=np.float64)
    assert p.size == NPARAM
    out, k = {}, 0
    for name, shape in SIZES:
        m = int(np.prod(shape))
        out[name] = p[k:k + m].reshape(shape)
        k += m
    return out


def init_params(seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SIZES:
        if name.startswith("b"):
            parts.append(np.zeros(int(np.prod(shape))))
        else:
            fan_in = shape[1] if len(shape) == 2 else shape[0]
            lim = 1.0 / np.sqrt(fan_in)
            parts.append(rng.uniform(-lim, lim, size=int(np.prod(shape))))
    return np.concatenate(parts)


def bf16_round(a) -> np.ndarray:
    """Round FP64 values to the nearest BF16 (ties to even), via FP32."""
    f = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> 16) & 1
    r = ((f + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, logtheta, norm):
    """Network output for a batch: returns (l~ [B], cache for ``backward``).
    norm = dict(mu_in[3], sd_in[3], mu_out, sd_out)."""
    P = unpack(p)
    X = np.atleast_2d(np.asarray(logtheta, dtype=np.float64))
    U = (X - np.asarray(norm["mu_in"])) / np.asarray(norm["sd_in"])
    H1 = np.tanh(U @ P["W1"].T + P["b1"])
    H2 = np.tanh(H1 @ P["W2"].T + P["b2"])
    O = H2 @ P["W3"] + P["b3"][0]
    return norm["mu_out"] + norm["sd_out"] * O, {"U": U, "H1": H1, "H2": H2, "O": O}


def loss_and_grad(p, logtheta, target, norm, bf16_products=False):
    """Standardized MSE of a batch and its gradient with respect to the flat
    parameter vector (chain rule, layer by layer).

    bf16_products=True takes the two 128-wide products of the network in the
    operand precision of a BF16 matrix unit: the hidden activations h1 are
    rounded to BF16 where they multiply W2 (forward) and dz2 (weight
    gradient), and the back-propagated dz2 is rounded to BF16 where it
    multiplies h1 and W2; every other value stays FP64 (the bias gradient of
    layer 2 sums the unrounded dz2)."""
    P = unpack(p)
    _, c = forward(p, logtheta, norm)
    H1 = c["H1"]
    H1p = H1
    if bf16_products:
        # the forward pass again with h1 rounded where it enters W2
        H1p = bf16_round(H1)
        c["H2"] = np.tanh(H1p @ P["W2"].T + P["b2"])
        c["O"] = c["H2"] @ P["W3"] + P["b3"][0]
    T = (np.asarray(target, dtype=np.float64) - norm["mu_out"]) / norm["sd_out"]
    B = T.size
    r = c["O"] - T
    loss = float(np.mean(r * r))
    g_o = 2.0 * r / B                                  # dloss/do, [B]
    g_W3 = c["H2"].T @ g_o                             # [128]
    g_b3 = np.array([g_o.sum()])
    g_z2 = np.outer(g_o, P["W3"]) * (1.0 - c["H2"] ** 2)  # [B,128]
    g_b2 = g_z2.sum(axis=0)
    g_z2p = bf16_round(g_z2) if bf16_products else g_z2
    g_W2 = g_z2p.T @ H1p                               # [128,128]
    g_h1 = g_z2p @ P["W2"]                             # [B,128]
    g_z1 = g_h1 * (1.0 - c["H1"] ** 2)
    g_W1 = g_z1.T @ c["U"]                             # [128,3]
    g_b1 = g_z1.sum(axis=0)
    grad = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_W3, g_b3])
    return loss, grad


def adam_step(p, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
