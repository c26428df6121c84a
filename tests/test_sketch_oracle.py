"""Pins for the oracle's randomized (sketch) compressor (oracle/hodlr_ref.py,
``sketch_compress``): its random signs and its accuracy.

* SplitMix64 against the reference generator's published outputs (seed 0 and
  seed 1234567, states advanced by the golden-ratio increment).
* The sign matrix is the bit pattern the key layout fixes (one word per 64
  columns, bit j mod 64, -1 for a set bit), rebuilt here bit by bit.
* An uncapped block is reproduced to its tolerance in the Frobenius norm
  (the reading of the truncation), with at least the optimal rank of the
  truncated SVD (numpy) and at most 20 % more; a rank-exact block (rank 3
  by construction) comes back with rank 3 and to rounding.
* The HODLR reference with this compressor gives the dense log det to
  the tolerance on a 2-D squared-exponential problem.
"""
import numpy as np
import pytest

import oracle
from oracle import hodlr_ref as hr


def test_splitmix64_matches_the_reference_outputs():
    def seq(seed, k):
        out, x = [], seed
        for _ in range(k):
            out.append(hr.splitmix64(x))
            x = (x + 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
        return out
    assert seq(0, 2) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]
    assert seq(1234567, 5) == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                               4593380528125082431, 16408922859458223821]


def test_sign_matrix_bit_layout():
    S = hr.sketch_signs(5, 1, 7, 70)
    for i in range(7):
        for j in range(70):
            w = hr.splitmix64(((2 * 5 + 1) << 40) | (i << 1) | (j // 64))
            assert S[i, j] == (-1.0 if (w >> (j % 64)) & 1 else 1.0)
    # roughly balanced and not constant along either axis
    assert abs(S.mean()) < 0.2 and len(np.unique(S[:, 0])) == 2 and len(np.unique(S[0])) == 2


def _block(n, side, ell, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, side, (n, 2))
    xs = x[hr.kd_order(x, 128)]
    m = n // 2
    return hr.kernel_block(0, xs[:m], xs[m:], 1.0, ell)


@pytest.mark.parametrize("n,side,ell,tol", [(2048, 0.25, 0.1, 1e-10), (2048, 0.25, 0.1, 1e-8),
                                            (2048, 0.1, 0.05, 1e-10), (1024, 1.0, 0.3, 1e-6)])
def test_uncapped_block_meets_its_tolerance(n, side, ell, tol):
    A = _block(n, side, ell, 7)
    U, V, capped = hr.sketch_compress(A, 0, 0, tol, 64)
    assert not capped
    sv = np.linalg.svd(A, compute_uv=False)
    k_opt = int(np.sum(sv > tol * sv[0]))
    err = np.linalg.norm(A - U @ V.T) / np.linalg.norm(A)
    assert err <= tol, err
    assert k_opt <= U.shape[1] <= int(np.ceil(1.2 * k_opt)) + 1, (U.shape[1], k_opt)


def test_exact_low_rank_block():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((300, 3)) @ rng.standard_normal((3, 400))
    U, V, capped = hr.sketch_compress(A, 2, 1, 1e-12, 16)
    assert U.shape[1] == 3 and not capped
    assert np.linalg.norm(A - U @ V.T) <= 1e-12 * np.linalg.norm(A)


def test_capped_block_reports_the_cap():
    A = _block(2048, 1.0, 0.2, 9)   # needs ~90 terms at 1e-10
    U, V, capped = hr.sketch_compress(A, 0, 0, 1e-10, 32)
    assert capped and U.shape[1] == 32


def test_hodlr_reference_with_sketch_matches_dense_logdet(oracle_lib):
    rng = np.random.default_rng(21)
    x = rng.uniform(0.0, 0.25, (2048, 2))
    y = rng.standard_normal(2048)
    R = hr.HodlrRef(x, 0, (1.0, 0.1), 1e-2, 128, 1e-10, max_rank=64, compress="sketch")
    assert R.capped == 0
    ref = oracle.gp_dense(x, y, 0, (1.0, 0.1), 1e-2)
    assert abs(R.logdet() - ref["logdet"]) <= 1e-9 * abs(ref["logdet"])
    # the quadratic form of an unrefined solve carries about tol ||K|| / sigma^2
    # (here ~1e-6) relative error in C^{-1} y, as with cross approximation
    ll = R.loglik(y)
    assert abs(ll["loglik"] - ref["loglik"]) <= 1e-7 * abs(ref["loglik"])
