"""The HODLR method's steps, written plainly in numpy (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The dense oracle gives the plain-definition result that the method
approximates to tolerance.  This module instead walks through the method
itself, in the paper's order, so that intermediate quantities (the tree,
the off-diagonal ranks, the per-node coupling determinants, the factor
list) can be pinned against what the mathematics fixes:

1. Ordering and tree (§3, k-d sorting; §3.2 pseudo-code sets the number of
   levels from the smallest block size).  Reading: L is the smallest level
   count with every leaf holding at most ``leaf`` points; a node of m points
   splits into a left child of floor(m/2) points and a right child of the rest;
   in D > 1 dimensions the node is sorted along coordinate (depth mod D)
   before the split, ties kept in input order.
2. Low-rank compression of every off-diagonal block K(alpha, beta) by
   (default) partially pivoted adaptive cross approximation (§3.1, "approximate
   partial-pivoted LU" with a sub-sampled error estimate).  Reading of the
   details the paper leaves out: start at the row of alpha next to the split
   (its last row); pivot column = first index of max |residual row|; a zero
   pivot marks the row used and moves to the unused row nearest the split
   (at most ``ZERO_RETRY`` times in a row); the stopping test after step k is
   ||u_k|| ||v_k|| <= tol ||S_k||_F with the Frobenius norm of the running
   approximation S_k updated incrementally; the next pivot row is the first
   index of max |u_k| over unused rows; at most min(max_rank, |alpha|, |beta|)
   terms.  Alternatively (compress="sketch") by the randomized two-sided
   sketch of ``sketch_compress``.
3. Leaf factor K_L: dense diagonal blocks C_lambda = K(lambda, lambda) +
   sigma^2 I, factored by Cholesky; their inverses applied to the rows of
   every off-diagonal basis that covers the leaf (§3.2 pseudo-code; §3.3).
4. Level by level from the leaves up: for node tau with children alpha,
   beta, the diagonal block is diag(C_alpha, C_beta) times
   I + diag(W~_alpha, W~_beta) [[0, W_beta^T], [W_alpha^T, 0]] (§3.2, the
   block low-rank update form), whose small coupling matrix is
   M = [[I, W_beta^T W~_beta], [W_alpha^T W~_alpha, I]].  Its inverse is
   applied by Sherman-Morrison-Woodbury to all remaining bases on tau's rows.
5. log det C = sum of leaf log-dets + sum of log det M_tau (§4: Sylvester's
   determinant theorem and multiplicativity of det over the factor list).
6. C^{-1} y applies the inverse factors leaves first (§3.2, the inverse of
   the factor list).

``panel32=True`` rounds every stored value of the applied bases W~ to FP32
(after the leaf solves and after each level's update) and keeps all
arithmetic in FP64: the storage precision of the mixed form, whose log-det
error this makes measurable on the CPU.  Not part of the paper's method.
"""
from __future__ import annotations

import math

import numpy as np

ZERO_RETRY = 8


# ----------------------------------------------------------------- kernels
def kernel_block(kind: int, xa: np.ndarray, xb: np.ndarray, a: float, ell: float) -> np.ndarray:
    """k(xa_i, xb_j) for point sets xa (m, D), xb (p, D): Table 1 / §5 kernels."""
    d = xa[:, None, :] - xb[None, :, :]
    r2 = np.sum(d * d, axis=-1)
    a2 = a * a
    if kind == 0:
        return a2 * np.exp(-r2 / (2.0 * ell * ell))
    if kind == 1:
        s = math.sqrt(3.0) * np.sqrt(r2) / ell
        return a2 * (1.0 + s) * np.exp(-s)
    if kind == 2:
        return a2 * np.exp(-np.sqrt(r2) / ell)
    if kind == 3:
        return np.full(r2.shape, a2)
    if kind == 4:
        return a2 / np.sqrt(1.0 + r2 / (ell * ell))
    raise ValueError("unknown kernel %r" % kind)


# -------------------------------------------------------- ordering and tree
def num_levels(n: int, leaf: int) -> int:
    """Smallest L >= 0 with ceil(n / 2^L) <= leaf."""
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    return L


def tree_nodes(n: int, L: int):
    """nodes[d] = list of (start, end) at depth d; left child gets floor(m/2)."""
    nodes = [[(0, n)]]
    for _ in range(L):
        nxt = []
        for (s, e) in nodes[-1]:
            m = s + (e - s) // 2
            nxt += [(s, m), (m, e)]
        nodes.append(nxt)
    return nodes


def kd_order(x: np.ndarray, leaf: int) -> np.ndarray:
    """Permutation putting points in k-d order: perm[k] = input index of the
    k-th ordered point.  1-D reduces to a stable sort."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    n, D = x.shape
    perm = np.arange(n, dtype=np.int64)
    L = num_levels(n, leaf)
    if D == 1:
        return np.argsort(x[:, 0], kind="stable").astype(np.int64)
    for d, level in enumerate(tree_nodes(n, L)[:L]):
        c = d % D
        for (s, e) in level:
            seg = perm[s:e]
            order = np.lexsort((seg, x[seg, c]))   # key c, ties by input index
            perm[s:e] = seg[order]
    return perm


# ------------------------------------------------------------------- ACA
def aca(row, col, m: int, nb: int, tol: float, max_rank: int):
    """Cross approximation A ~ U V^T of an m x nb block given row(i) -> A[i, :]
    and col(j) -> A[:, j].  Returns (U (m x r), V (nb x r), capped)."""
    U, V = [], []
    # a block never needs more terms than its size; only the user's cap counts as "capped"
    full = min(m, nb)
    user_cap = max_rank < full
    max_rank = min(max_rank, full)
    if m == 0 or nb == 0 or max_rank <= 0:
        return np.zeros((m, 0)), np.zeros((nb, 0)), False
    used = np.zeros(m, dtype=bool)
    istar = m - 1
    s2 = 0.0
    zeros_in_row = 0
    capped = False
    while True:
        v = np.array(row(istar), dtype=np.float64)
        for ul, vl in zip(U, V):
            v -= ul[istar] * vl
        jstar = int(np.argmax(np.abs(v)))
        delta = v[jstar]
        used[istar] = True
        if delta == 0.0:
            zeros_in_row += 1
            if zeros_in_row > ZERO_RETRY or used.all():
                break
            istar = int(np.nonzero(~used)[0][-1])
            continue
        zeros_in_row = 0
        u = np.array(col(jstar), dtype=np.float64)
        for ul, vl in zip(U, V):
            u -= vl[jstar] * ul
        u /= delta
        s2 += float(u @ u) * float(v @ v)
        for ul, vl in zip(U, V):
            s2 += 2.0 * float(ul @ u) * float(vl @ v)
        U.append(u)
        V.append(v)
        if math.sqrt(float(u @ u)) * math.sqrt(float(v @ v)) <= tol * math.sqrt(max(s2, 0.0)):
            break
        if len(U) >= max_rank:
            capped = user_cap
            break
        if used.all():
            break
        au = np.abs(u)
        au[used] = -1.0
        istar = int(np.argmax(au))
    r = len(U)
    Um = np.stack(U, axis=1) if r else np.zeros((m, 0))
    Vm = np.stack(V, axis=1) if r else np.zeros((nb, 0))
    return Um, Vm, capped


# ------------------------------------------------------------ factorization
# ---------------------------------------------------- randomized compression
# Second compressor of §3.1's list of algebraic low-rank methods: a two-sided
# randomized sketch (generalized Nystrom).  For A = K(alpha, beta) (m x nb):
#   X (nb x s) and Y (m x s') random signs, s = min(cap + 16, m, nb),
#   s' = min(s + 8, m);  AX, Y^T A and the core C = Y^T A X;
#   A ~ AX C^+ Y^T A with the pseudo-inverse truncated to the k singular
#   values of C above SKETCH_CUT * tol * sigma_1(C) (capped when k > cap):
#   U = AX Q_k S_k^{-1/2},  V = (Y^T A)^T P_k S_k^{-1/2}  (C = P S Q^T).
# Readings (the paper names randomized methods without fixing one): signs
# from SplitMix64 of a per-entry key, the oversampling 16 / 8, and the cut
# at tol / 10, which kept ||A - U V^T||_F <= tol ||A||_F on the tested 2-D
# squared-exponential blocks where a cut at tol did not.
SKETCH_OVER_X = 16
SKETCH_OVER_Y = 8
SKETCH_CUT = 0.1
_M64 = (1 << 64) - 1


def splitmix64(key: int) -> int:
    """SplitMix64's output for state `key` (Steele, Lea, Flood 2014; Vigna's
    public-domain reference): the state advances by the golden-ratio
    increment, then two xor-shift-multiply rounds and a final xor-shift."""
    z = (key + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def sketch_signs(node: int, side: int, nrows: int, ns: int) -> np.ndarray:
    """(nrows x ns) matrix of +-1: entry (i, j) is -1 when bit j mod 64 of
    splitmix64(((2 node + side) << 40) | (i << 1) | (j >> 6)) is set.
    side 0: X over beta's points, 1: Y over alpha's points; node = heap index."""
    out = np.empty((nrows, ns), dtype=np.float64)
    for i in range(nrows):
        words = [splitmix64(((2 * node + side) << 40) | (i << 1) | b) for b in range((ns + 63) // 64)]
        for j in range(ns):
            out[i, j] = -1.0 if (words[j >> 6] >> (j & 63)) & 1 else 1.0
    return out


def sketch_compress(A: np.ndarray, depth: int, idx: int, tol: float, cap: int):
    """Returns (U, V, capped) for block A of the depth-`depth` node number
    `idx` (heap index 2^depth - 1 + idx)."""
    m, nb = A.shape
    h = (1 << depth) - 1 + idx
    s = min(cap + SKETCH_OVER_X, m, nb)
    if s <= 0 or cap <= 0:
        return np.zeros((m, 0)), np.zeros((nb, 0)), False
    sp = min(s + SKETCH_OVER_Y, m)
    X = sketch_signs(h, 0, nb, s)
    Y = sketch_signs(h, 1, m, sp)
    AX = A @ X
    YA = Y.T @ A
    C = Y.T @ AX
    P, S, Qt = np.linalg.svd(C, full_matrices=False)
    k = int(np.sum(S > SKETCH_CUT * tol * S[0])) if S.size and S[0] > 0 else 0
    capped = k > cap
    k = min(k, cap)
    U = AX @ (Qt[:k].T / np.sqrt(S[:k]))
    V = YA.T @ (P[:, :k] / np.sqrt(S[:k]))
    return U, V, capped


class HodlrRef:
    """Plain FP64 HODLR factorization of C = sigma^2 I + K on ordered points."""

    def __init__(self, x, kind, theta, sigma2, leaf, tol, max_rank=64, presorted=False,
                 compress="aca", panel32=False):
        self.panel32 = bool(panel32)
        x = np.asarray(x, dtype=np.float64)
        if x.ndim == 1:
            x = x.reshape(-1, 1)
        self.n, self.dim = x.shape
        self.perm = np.arange(self.n) if presorted else kd_order(x, leaf)
        self.xs = x[self.perm]
        self.kind, self.theta, self.sigma2 = kind, tuple(theta), float(sigma2)
        self.leaf, self.tol, self.max_rank = leaf, tol, max_rank
        self.L = num_levels(self.n, leaf)
        self.nodes = tree_nodes(self.n, self.L)
        self._compress(compress)
        self._factor()

    # K restricted to index ranges of the ordered points
    def K(self, rs, cs):
        a, ell = self.theta
        return kernel_block(self.kind, self.xs[rs[0]:rs[1]], self.xs[cs[0]:cs[1]], a, ell)

    def _compress(self, method):
        """W[d] = list over depth-d nodes of their bases (rows of node x r_parent)."""
        a, ell = self.theta
        self.ranks = []       # ranks[d][i] for non-leaf node i at depth d
        self.capped = 0
        self.W = [None] + [[None] * len(self.nodes[d]) for d in range(1, self.L + 1)]
        for d in range(self.L):
            rk = []
            for i, (s, e) in enumerate(self.nodes[d]):
                m = s + (e - s) // 2
                xa, xb = self.xs[s:m], self.xs[m:e]
                if method == "aca":
                    U, V, cap = aca(lambda ii: kernel_block(self.kind, xa[ii:ii + 1], xb, a, ell)[0],
                                    lambda jj: kernel_block(self.kind, xa, xb[jj:jj + 1], a, ell)[:, 0],
                                    m - s, e - m, self.tol, self.max_rank)
                    self.capped += int(cap)
                elif method == "sketch":
                    A = kernel_block(self.kind, xa, xb, a, ell)
                    U, V, cap = sketch_compress(A, d, i, self.tol, self.max_rank)
                    self.capped += int(cap)
                else:   # truncated SVD (optimal rank, used only in tests)
                    A = kernel_block(self.kind, xa, xb, a, ell)
                    Us, sv, Vt = np.linalg.svd(A, full_matrices=False)
                    r = int(np.sum(sv > self.tol * (sv[0] if sv.size else 0.0)))
                    U, V = Us[:, :r] * sv[:r], Vt[:r].T
                self.W[d + 1][2 * i] = U
                self.W[d + 1][2 * i + 1] = V
                rk.append(U.shape[1])
            self.ranks.append(rk)

    def _factor(self):
        L, n = self.L, self.n
        # leaves
        self.G = []
        self.leaf_logdet = []
        for (s, e) in self.nodes[L]:
            C = self.K((s, e), (s, e)) + self.sigma2 * np.eye(e - s)
            G = np.linalg.cholesky(C) if e > s else np.zeros((0, 0))
            self.G.append(G)
            self.leaf_logdet.append(2.0 * float(np.sum(np.log(np.diag(G)))))
        # W~ starts as a copy of W, then gets C_leaf^{-1} on every leaf's rows
        self.Wt = [None] + [[w.copy() for w in self.W[d]] for d in range(1, L + 1)]
        for d in range(1, L + 1):
            for j, (s, e) in enumerate(self.nodes[d]):
                for li, (ls, le) in enumerate(self.nodes[L]):
                    if ls >= s and le <= e and le > ls:
                        blk = self.Wt[d][j][ls - s:le - s]
                        self.Wt[d][j][ls - s:le - s] = self._store(self._leaf_solve(li, blk))
        # levels, from the leaves' parents up to the root
        self.M = [None] * L
        self.node_logdet = [None] * L
        for d in range(L - 1, -1, -1):
            self.M[d] = []
            self.node_logdet[d] = []
            for i, (s, e) in enumerate(self.nodes[d]):
                mid = s + (e - s) // 2
                Wa, Wb = self.W[d + 1][2 * i], self.W[d + 1][2 * i + 1]
                Ta, Tb = self.Wt[d + 1][2 * i], self.Wt[d + 1][2 * i + 1]
                r = Wa.shape[1]
                P = Wb.T @ Tb
                Q = Wa.T @ Ta
                Mt = np.block([[np.eye(r), P], [Q, np.eye(r)]])
                sign, ldm = np.linalg.slogdet(Mt) if r else (1.0, 0.0)
                if sign <= 0:
                    raise np.linalg.LinAlgError("coupling determinant not positive")
                self.M[d].append(Mt)
                self.node_logdet[d].append(float(ldm))
                # remaining bases on tau's rows: ancestors at depths 1..d
                for j in range(1, d + 1):
                    anc = [(jj, se) for jj, se in enumerate(self.nodes[j])
                           if se[0] <= s and se[1] >= e]
                    jj, (as_, ae) = anc[0]
                    X = self.Wt[j][jj]
                    Xa = X[s - as_:mid - as_]
                    Xb = X[mid - as_:e - as_]
                    if r:
                        S = np.linalg.solve(Mt, np.vstack([Wb.T @ Xb, Wa.T @ Xa]))
                        X[s - as_:mid - as_] = self._store(Xa - Ta @ S[:r])
                        X[mid - as_:e - as_] = self._store(Xb - Tb @ S[r:])

    def _store(self, A):
        """A value of W~ as stored: FP64, or rounded to FP32 with panel32."""
        return A.astype(np.float32).astype(np.float64) if self.panel32 else A

    def _leaf_solve(self, li, B):
        G = self.G[li]
        z = np.linalg.solve(G, B)
        return np.linalg.solve(G.T, z)

    # ---------------------------------------------------------------- results
    def logdet(self) -> float:
        parts = list(self.leaf_logdet)
        for d in range(self.L):
            parts += self.node_logdet[d]
        return float(math.fsum(parts))

    def solve_ordered(self, b: np.ndarray) -> np.ndarray:
        """C^{-1} b for b in the tree (ordered) index space."""
        L = self.L
        z = np.array(b, dtype=np.float64, copy=True)
        for li, (s, e) in enumerate(self.nodes[L]):
            if e > s:
                z[s:e] = self._leaf_solve(li, z[s:e])
        for d in range(L - 1, -1, -1):
            for i, (s, e) in enumerate(self.nodes[d]):
                mid = s + (e - s) // 2
                Wa, Wb = self.W[d + 1][2 * i], self.W[d + 1][2 * i + 1]
                Ta, Tb = self.Wt[d + 1][2 * i], self.Wt[d + 1][2 * i + 1]
                r = Wa.shape[1]
                if r == 0:
                    continue
                S = np.linalg.solve(self.M[d][i], np.concatenate([Wb.T @ z[mid:e], Wa.T @ z[s:mid]]))
                z[s:mid] -= Ta @ S[:r]
                z[mid:e] -= Tb @ S[r:]
        return z

    def solve(self, y) -> np.ndarray:
        """C^{-1} y in the caller's order."""
        y = np.asarray(y, dtype=np.float64)
        z = self.solve_ordered(y[self.perm])
        out = np.empty_like(z)
        out[self.perm] = z
        return out

    def loglik(self, y):
        alpha = self.solve(y)
        q = float(np.dot(y, alpha))
        ld = self.logdet()
        return {"logdet": ld, "quad": q,
                "loglik": -0.5 * q - 0.5 * ld - 0.5 * self.n * math.log(2.0 * math.pi),
                "alpha": alpha}

    def factor_matrices(self):
        """Dense factor list [K_L, B_{L-1}, ..., B_0] in ordered index space,
        whose product approximates C (the factorization K = K_k ... K_0 of §3.2)."""
        n, L = self.n, self.L
        KL = np.zeros((n, n))
        for li, (s, e) in enumerate(self.nodes[L]):
            KL[s:e, s:e] = self.G[li] @ self.G[li].T
        out = [KL]
        for d in range(L - 1, -1, -1):
            B = np.eye(n)
            for i, (s, e) in enumerate(self.nodes[d]):
                mid = s + (e - s) // 2
                Wa, Wb = self.W[d + 1][2 * i], self.W[d + 1][2 * i + 1]
                Ta, Tb = self.Wt[d + 1][2 * i], self.Wt[d + 1][2 * i + 1]
                B[s:mid, mid:e] += Ta @ Wb.T
                B[mid:e, s:mid] += Tb @ Wa.T
            out.append(B)
        return out
