"""Gradient of the GP log-likelihood in its hyperparameters, from dense
matrices (TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may use anything under ``oracle/``).

The likelihood is Eq. (1) of the paper with C = sigma^2 I + K(theta),
theta = (a, l) (§2.1; the kernels of Table 1 and §5 as in ``dense_oracle.c``).
Its hyperparameter fits (§2.3) iterate on the likelihood; differentiating
Eq. (1) gives, for each parameter p with dC/dp = C_p,

    dL/dp = 1/2 alpha^T C_p alpha - 1/2 tr(C^{-1} C_p),   alpha = C^{-1} y,

written out here with a dense Cholesky factor and the explicit inverse:
    C_a      = 2 K / a                      (K is proportional to a^2),
    C_sigma2 = I,
    C_l      = a^2 dk/dl entrywise, with r the distance between the points:
        squared exponential     k = exp(-r^2 / (2 l^2)),   dk/dl = k r^2 / l^3
        Matern nu = 3/2         k = (1 + s) exp(-s), s = sqrt(3) r / l,
                                dk/dl = s^2 exp(-s) / l
        exponential             k = exp(-r / l),           dk/dl = k r / l^2
        constant                k = 1,                     dk/dl = 0
        inverse multiquadric    k = (1 + r^2 / l^2)^(-1/2),
                                dk/dl = (r^2 / l^3) (1 + r^2 / l^2)^(-3/2)

Pinned in tests/test_grad_oracle.py against an eigendecomposition route for
the a and sigma^2 parts (closed form in the eigenvalues of the unit-amplitude
kernel matrix) and against high-order finite differences of the dense
likelihood for the l part.
"""
from __future__ import annotations

import numpy as np

from . import dense_matrix, gp_dense, _pts

K_SE, K_MATERN32, K_EXP, K_CONST, K_IMQ = 0, 1, 2, 3, 4


def _dist(x):
    x = _pts(x)
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(axis=2)
    return np.sqrt(d2), d2


def dkernel_dl(x, kind: int, a: float, ell: float) -> np.ndarray:
    """a^2 dk/dl between all pairs of points (the matrix C_l)."""
    r, r2 = _dist(x)
    a2 = a * a
    if kind == K_SE:
        return a2 * np.exp(-r2 / (2.0 * ell * ell)) * r2 / ell ** 3
    if kind == K_MATERN32:
        s = np.sqrt(3.0) * r / ell
        return a2 * s * s * np.exp(-s) / ell
    if kind == K_EXP:
        return a2 * np.exp(-r / ell) * r / (ell * ell)
    if kind == K_CONST:
        return np.zeros_like(r)
    if kind == K_IMQ:
        u = 1.0 + r2 / (ell * ell)
        return a2 * (r2 / ell ** 3) * u ** -1.5
    raise ValueError("unknown kernel %d" % kind)


def gp_dense_grad(x, y, kind: int, theta, sigma2: float):
    """Returns dict(loglik, grad = [dL/da, dL/dl, dL/dsigma2])."""
    x = _pts(x)
    y = np.asarray(y, dtype=np.float64).ravel()
    n = x.shape[0]
    a, ell = float(theta[0]), float(theta[1])
    C = dense_matrix(x, kind, (a, ell), sigma2)
    K = C - sigma2 * np.eye(n)
    G = np.linalg.cholesky(C)
    Ginv = np.linalg.inv(G)
    Cinv = Ginv.T @ Ginv
    alpha = Cinv @ y
    mats = [2.0 * K / a, dkernel_dl(x, kind, a, ell), np.eye(n)]
    grad = [0.5 * alpha @ (Cp @ alpha) - 0.5 * np.sum(Cinv * Cp) for Cp in mats]
    return {"loglik": gp_dense(x, y, kind, (a, ell), sigma2)["loglik"], "grad": np.array(grad)}
