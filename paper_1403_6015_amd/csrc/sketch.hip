// Randomized compression of the off-diagonal blocks, the alternative to
// cross approximation among §3.1's algebraic low-rank methods: a two-sided
// sketch (generalized Nystrom).  For the block A = K(alpha, beta) of node
// tau (m x nb, entries evaluated on the fly from the ordered points):
//   s = min(cap + SK_OVER_X, m, nb) columns of random signs X (nb x s) and
//   s' = min(s + SK_OVER_Y, m) of Y (m x s');
//   A X (alpha's rows) and A^T Y (beta's rows; the kernel is symmetric, so
//   the same code with the children swapped), each entry of A evaluated once
//   per sketch, on FP64 MFMA;
//   the core C = Y^T A X (s' x s), summed from per-64-row partials;
//   C = P S Q^T by one-sided Jacobi (Hestenes) in one work-group per node;
//   k = the singular values above SK_CUT tol S_1 (capped at cap), and
//   U = A X Q_k S_k^{-1/2} into alpha's rows and V = A^T Y P_k S_k^{-1/2}
//   into beta's rows of the depth-(d+1) panel, so A ~ U V^T as after cross
//   approximation and the rest of the factorization is unchanged.
// Signs: entry (i, j) of the sketch on side t (0: X over beta's points, 1: Y
// over alpha's points) of node h is -1 when bit j mod 64 of
// SplitMix64(((2h + t) << 40) | (i << 1) | (j >> 6)) is set; SplitMix64 is
// Steele, Lea and Flood's generator (OOPSLA 2014), its output function as in
// Vigna's public-domain reference.  Levels are compressed one at a time
// (their sketches share one buffer), four launches each.
#include "common.h"

namespace hodlr {

constexpr double SK_CUT = 0.1;   // truncation at SK_CUT * tol of the core's largest singular value
constexpr int SK_SWEEPS = 40;
typedef double sk_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t sk_mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct SketchArgs {
    KParams kp;
    const double *x;
    int64_t n;
    const int64_t *start, *end;
    const Chunk *chunks;   // the level's 64-row chunks
    const int *abase, *acnt;
    int64_t node0;         // heap index of the level's first node
    int cap;
    double tol;
    double *sk;            // n x SK_SPMAX, column-major: the level's sketch rows
    double *part;          // per alpha chunk: SK_SPMAX x SK_SMAX partial core (row-major)
    double *core;          // per node of the level: SK_SPMAX x SK_SMAX
    double *fac;           // per node: R (SK_SMAX x SK_CAP_MAX), then L (SK_SPMAX x SK_CAP_MAX)
    int *rank, *status;    // per heap node
    double *W;
    int64_t col0;          // first panel column of depth d+1
};

constexpr int64_t SK_CORE = (int64_t)SK_SPMAX * SK_SMAX;
constexpr int64_t SK_FAC = (int64_t)(SK_SMAX + SK_SPMAX) * SK_CAP_MAX;

// the node's split and sketch widths (s = 0: nothing to compress)
__device__ __forceinline__ void sk_sizes(const SketchArgs &S, int64_t h, int64_t &lo, int64_t &mid,
                                         int64_t &hi, int &s, int &sp)
{
    lo = S.start[h];
    hi = S.end[h];
    mid = lo + (hi - lo) / 2;
    int64_t t = S.cap > 0 ? (int64_t)S.cap + SK_OVER_X : 0;
    t = t < mid - lo ? t : mid - lo;
    t = t < hi - mid ? t : hi - mid;
    s = (int)t;
    sp = s > 0 ? (int)((t + SK_OVER_Y) < (mid - lo) ? t + SK_OVER_Y : mid - lo) : 0;
}

// sign of sketch entry (i, j) on side t of node h, from its word
__device__ __forceinline__ double sk_sign(uint64_t w, int j)
{
    return ((w >> (j & 63)) & 1ull) ? -1.0 : 1.0;
}

// One 64-row chunk of one child: its rows of A X (alpha) or A^T Y (beta),
// 16 rows per wave, NT tiles of 16 sketch columns.  Lane (r, q) evaluates
// A[row r][column c0 + q] (the MFMA's A operand) and the signs of column
// c0 + q (its B operand); it ends holding rows q + 4u of sketch columns
// 16 t + r.  Alpha chunks also write their partial core Y^T (A X) over their
// 64 rows, with A X staged in LDS.
template <int NT>
__global__ __launch_bounds__(256) void sketch_kernel(SketchArgs S)
{
    const Chunk ch = S.chunks[blockIdx.x];
    const int64_t h = ch.node;
    int64_t lo, mid, hi;
    int s, sp;
    sk_sizes(S, h, lo, mid, hi, s, sp);
    if (s == 0)
        return;   // the whole work-group
    __shared__ double sAX[SK_ROWS][SK_SMAX + 1];
    const int side = ch.side;
    const int nsamp = side ? sp : s;
    const int64_t c_lo = side ? lo : mid, c_hi = side ? mid : hi;
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6), r = lane & 15, q = lane >> 4;
    const int64_t n = S.n;
    const int64_t wr0 = ch.lo + 16 * wid;
    const int64_t gi = wr0 + r;
    const bool rok = gi < ch.hi;
    const uint64_t kb = (uint64_t)(2 * h + side) << 40;
    const bool two = nsamp > 64;
    sk_d4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        acc[t] = sk_d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t c0 = c_lo; c0 < c_hi; c0 += 4) {
        const int64_t gc = c0 + q;
        const bool cok = gc < c_hi;
        const double a = (rok && cok) ? kentry(S.kp, S.x, n, gi, gc) : 0.0;
        const uint64_t ci = (uint64_t)(cok ? gc - c_lo : 0);
        const uint64_t w0 = sk_mix(kb | (ci << 1));
        const uint64_t w1 = two ? sk_mix(kb | (ci << 1) | 1ull) : 0ull;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = 16 * t + r;
            const double b = (cok && j < nsamp) ? sk_sign(j < 64 ? w0 : w1, j) : 0.0;
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = wr0 + q + 4 * u;
            const int j = 16 * t + r;
            if (row < ch.hi && j < nsamp)
                S.sk[(int64_t)j * n + row] = acc[t][u];
        }
    if (side != 0)
        return;   // the whole work-group
    // partial core over this chunk's rows: C[a][b] = sum_i Y[i][a] (A X)[i][b]
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int lr = 16 * wid + q + 4 * u, j = 16 * t + r;
            if (j < SK_SMAX)
                sAX[lr][j] = (wr0 + q + 4 * u < ch.hi && j < s) ? acc[t][u] : 0.0;
        }
    __syncthreads();
    const int ta_n = (sp + 15) / 16, tb_n = (s + 15) / 16;
    const uint64_t ky = (uint64_t)(2 * h + 1) << 40;
    double *out = S.part + (int64_t)ch.part * SK_CORE;
    for (int tt = wid; tt < ta_n * tb_n; tt += 4) {
        const int ta = tt / tb_n, tb = tt % tb_n;
        const int ai = 16 * ta + r;
        sk_d4 c = {0.0, 0.0, 0.0, 0.0};
        for (int ks = 0; ks < SK_ROWS / 4; ++ks) {
            const int lr = 4 * ks + q;
            const int64_t grow = ch.lo + lr;
            double ya = 0.0;
            if (grow < ch.hi && ai < sp)
                ya = sk_sign(sk_mix(ky | ((uint64_t)(grow - lo) << 1) | (uint64_t)(ai >> 6)), ai);
            const double bx = sAX[lr][16 * tb + r];
            c = __builtin_amdgcn_mfma_f64_16x16x4f64(ya, bx, c, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int a = 16 * ta + q + 4 * u, b = 16 * tb + r;
            if (a < sp && b < s)
                out[a * SK_SMAX + b] = c[u];
        }
    }
}

// core of each node of the level: the sum of its alpha chunks' partials, in
// chunk order (one thread per entry)
__global__ __launch_bounds__(256) void sk_core_sum_kernel(SketchArgs S)
{
    const int64_t loc = blockIdx.x;
    const int64_t h = S.node0 + loc;
    const int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x;
    if (e >= SK_CORE)
        return;
    int64_t lo, mid, hi;
    int s, sp;
    sk_sizes(S, h, lo, mid, hi, s, sp);
    const int a = (int)(e / SK_SMAX), b = (int)(e % SK_SMAX);
    double v = 0.0;
    if (a < sp && b < s) {
        const int c0 = S.abase[loc], c1 = c0 + S.acnt[loc];
        for (int c = c0; c < c1; ++c)
            v += S.part[(int64_t)c * SK_CORE + e];
    }
    S.core[loc * SK_CORE + e] = v;
}

// SVD of each node's core C (sp x s, one work-group per node), the rank and
// the maps R = Q_k S_k^{-1/2} (for A X) and L = P_k S_k^{-1/2} (for A^T Y):
//   1. C Pi = Q R by Householder QR with column pivoting (largest remaining
//      column norm, recomputed every step; first index on ties); the
//      reflectors (v_k with v_kk = 1, and tau_k on the diagonal) go to the
//      node's core slot in HBM, which the core no longer needs;
//   2. one-sided Jacobi (Hestenes) on the columns of M = R^T with the
//      rotations accumulated in V: M V = W S.  Pivoted QR first makes the
//      sweeps few (Drmac and Veselic); without it a core whose singular values
//      span 16 decades took 24 sweeps and more.  Columns are paired by the
//      circle method (s/2 disjoint pairs per round, one wave per pair); a pair
//      is rotated when |c_p . c_q| > 1e-15 |c_p| |c_q|, unless one column has
//      fallen below SK_NEGL times the truncation level (SK_CUT tol ||C||_F):
//      leaving such a pair moves the larger column by at most that much, far
//      below what is truncated.  Sweeps end when no pair was rotated (at most
//      SK_SWEEPS);
//   3. singular values = the rotated columns' norms (ordered, ties to the
//      smaller index), k = those above SK_CUT tol S_1 (at most the cap);
//      C = (Q V) S (Pi W)^T, so R = Pi W_k S_k^{-1/2} (row Pi(i) of R is row
//      i of the rotated M over S^{3/2}) and L = Q V_k S_k^{-1/2}, formed by
//      applying the reflectors to [V_k S_k^{-1/2}; 0].
constexpr int SK_SVD_TH = 1024;
constexpr double SK_NEGL = 1e-3;

__global__ __launch_bounds__(SK_SVD_TH) void sk_svd_kernel(SketchArgs S)
{
    const int64_t loc = blockIdx.x;
    const int64_t h = S.node0 + loc;
    int64_t lo, mid, hi;
    int s, sp;
    sk_sizes(S, h, lo, mid, hi, s, sp);
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int NW = SK_SVD_TH / 64;
    if (s == 0) {
        if (tid == 0) {
            S.rank[h] = 0;
            S.status[h] = ACA_CONVERGED;
        }
        return;
    }
    constexpr int LA = SK_SPMAX + 1, LV = SK_SMAX + 1;
    __shared__ double sA[SK_SMAX * LA];   // column j at sA + j * LA: C, then R / M, then Q's input
    __shared__ double sV[SK_SMAX * LV];   // column j at sV + j * LV (s rows)
    __shared__ double snrm[SK_SMAX], stau[SK_SMAX], sig[SK_SMAX], sfro[NW];
    __shared__ int perm[SK_SMAX], ord[SK_SMAX];
    __shared__ int s_rot, s_k, s_p;
    double *hh = S.core + loc * SK_CORE;   // reflectors: v_k at hh[i * SK_SMAX + k], i > k
    double fro = 0.0;
    for (int e = tid; e < s * sp; e += SK_SVD_TH) {
        const int j = e / sp, i = e % sp;
        const double v = hh[i * SK_SMAX + j];
        sA[j * LA + i] = v;
        fro += v * v;
    }
    fro = wave_sum(fro);
    if (lane == 0)
        sfro[wid] = fro;
    for (int j = tid; j < s; j += SK_SVD_TH)
        perm[j] = j;
    __syncthreads();
    double fro2 = 0.0;
    for (int w = 0; w < NW; ++w)
        fro2 += sfro[w];
    // 1. pivoted QR
    const int K = s < sp ? s : sp;
    for (int k = 0; k < K; ++k) {
        for (int j = k + wid; j < s; j += NW) {
            double v = 0.0;
            for (int i = k + lane; i < sp; i += 64)
                v += sA[j * LA + i] * sA[j * LA + i];
            v = wave_sum(v);
            if (lane == 0)
                snrm[j] = v;
        }
        __syncthreads();
        if (tid == 0) {
            int p = k;
            for (int j = k + 1; j < s; ++j)
                if (snrm[j] > snrm[p])
                    p = j;
            s_p = p;
            const int t = perm[k];
            perm[k] = perm[p];
            perm[p] = t;
        }
        __syncthreads();
        const int p = s_p;
        if (p != k)
            for (int i = tid; i < sp; i += SK_SVD_TH) {
                const double t = sA[k * LA + i];
                sA[k * LA + i] = sA[p * LA + i];
                sA[p * LA + i] = t;
            }
        __syncthreads();
        if (wid == 0) {   // the reflector of column k
            double x0 = sA[k * LA + k], v = 0.0;
            for (int i = k + lane; i < sp; i += 64)
                v += sA[k * LA + i] * sA[k * LA + i];
            const double nx = sqrt(wave_sum(v));
            double tau = 0.0, beta = x0, scale = 0.0;
            if (nx > 0.0) {
                beta = x0 >= 0.0 ? -nx : nx;
                tau = (beta - x0) / beta;
                scale = 1.0 / (x0 - beta);
            }
            for (int i = k + 1 + lane; i < sp; i += 64)
                sA[k * LA + i] *= scale;
            if (lane == 0) {
                sA[k * LA + k] = beta;
                stau[k] = tau;
            }
        }
        __syncthreads();
        const double tau = stau[k];
        for (int j = k + 1 + wid; j < s; j += NW) {   // H_k applied to the columns right of k
            double w = 0.0;
            for (int i = k + lane; i < sp; i += 64)
                w += (i == k ? 1.0 : sA[k * LA + i]) * sA[j * LA + i];
            w = wave_sum(w) * tau;
            for (int i = k + lane; i < sp; i += 64)
                sA[j * LA + i] -= w * (i == k ? 1.0 : sA[k * LA + i]);
        }
        __syncthreads();
    }
    // reflectors to the core slot; M = R^T in place (s x s, zero above the
    // diagonal and below row s)
    for (int e = tid; e < K * sp; e += SK_SVD_TH) {
        const int k = e / sp, i = e % sp;
        if (i > k)
            hh[i * SK_SMAX + k] = sA[k * LA + i];
        else if (i == k)
            hh[i * SK_SMAX + k] = stau[k];
    }
    __syncthreads();
    for (int e = tid; e < s * sp; e += SK_SVD_TH) {
        const int j = e / sp, i = e % sp;   // entry (i, j) of the new M, from R(j, i)
        if (i < j || i >= s)
            continue;
        if (i == j)
            continue;   // the diagonal stays
        // i > j: M(i, j) = R(j, i), stored at column i, row j
        sA[j * LA + i] = sA[i * LA + j];
    }
    __syncthreads();
    for (int e = tid; e < s * sp; e += SK_SVD_TH) {
        const int j = e / sp, i = e % sp;
        if (i < j || i >= s)
            if (!(i == j))
                sA[j * LA + i] = 0.0;
    }
    for (int e = tid; e < s * s; e += SK_SVD_TH) {
        const int j = e / s, i = e % s;
        sV[j * LV + i] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    // 2. Jacobi on the columns of M
    const double negl = SK_NEGL * SK_CUT * S.tol;
    const double negl2 = negl * negl * fro2;
    const int ns = (s + 1) & ~1;   // even; index s (odd s) is an absent column
    for (int sweep = 0; sweep < SK_SWEEPS; ++sweep) {
        if (tid == 0)
            s_rot = 0;
        __syncthreads();
        for (int round = 0; round < ns - 1; ++round) {
            for (int pr = wid; pr < ns / 2; pr += NW) {
                const int p = pr == 0 ? 0 : (pr - 1 + round) % (ns - 1) + 1;
                const int qq = (ns - 2 - pr + round) % (ns - 1) + 1;
                if (p >= s || qq >= s)
                    continue;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = lane; i < s; i += 64) {
                    const double cp = sA[p * LA + i], cq = sA[qq * LA + i];
                    al += cp * cp;
                    be += cq * cq;
                    ga += cp * cq;
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                if (fabs(ga) > 1e-15 * sqrt(al * be) && fmin(al, be) > negl2) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                    for (int i = lane; i < s; i += 64) {
                        const double cp = sA[p * LA + i], cq = sA[qq * LA + i];
                        sA[p * LA + i] = cs * cp - sn * cq;
                        sA[qq * LA + i] = sn * cp + cs * cq;
                        const double vp = sV[p * LV + i], vq = sV[qq * LV + i];
                        sV[p * LV + i] = cs * vp - sn * vq;
                        sV[qq * LV + i] = sn * vp + cs * vq;
                    }
                    if (lane == 0)
                        s_rot = 1;
                }
            }
            __syncthreads();
        }
        const int rot = s_rot;
        __syncthreads();   // everyone has read s_rot before it is reset
        if (!rot)
            break;
    }
    // 3. singular values, order, rank
    for (int j = wid; j < s; j += NW) {
        double v = 0.0;
        for (int i = lane; i < s; i += 64)
            v += sA[j * LA + i] * sA[j * LA + i];
        v = wave_sum(v);
        if (lane == 0)
            sig[j] = sqrt(v);
    }
    __syncthreads();
    double smax = 0.0;
    for (int j = 0; j < s; ++j)
        smax = fmax(smax, sig[j]);
    if (tid < s) {
        const double v = sig[tid];
        int rk = 0;
        for (int j = 0; j < s; ++j)
            rk += (sig[j] > v || (sig[j] == v && j < tid)) ? 1 : 0;
        ord[rk] = tid;
    }
    if (tid == 0) {
        int k = 0;
        if (smax > 0.0)
            for (int j = 0; j < s; ++j)
                k += (sig[j] > SK_CUT * S.tol * smax) ? 1 : 0;
        const bool capped = k > S.cap;
        k = capped ? S.cap : k;
        s_k = k;
        S.rank[h] = k;
        S.status[h] = capped ? ACA_CAPPED : ACA_CONVERGED;
    }
    __syncthreads();
    const int k = s_k;
    double *R = S.fac + loc * SK_FAC;
    double *Lm = R + SK_SMAX * SK_CAP_MAX;
    for (int e = tid; e < s * k; e += SK_SVD_TH) {
        const int i = e / k, l = e % k, j = ord[l];
        R[perm[i] * SK_CAP_MAX + l] = sA[j * LA + i] / (sig[j] * sqrt(sig[j]));
    }
    __syncthreads();   // sA is reused for Q's input below
    for (int e = tid; e < k * sp; e += SK_SVD_TH) {
        const int l = e / sp, i = e % sp, j = ord[l];
        sA[l * LA + i] = i < s ? sV[j * LV + i] / sqrt(sig[j]) : 0.0;
    }
    __syncthreads();
    for (int kk = K - 1; kk >= 0; --kk) {   // L = H_0 ... H_{K-1} [V_k S_k^{-1/2}; 0]
        const double tau = hh[kk * SK_SMAX + kk];
        for (int l = wid; l < k; l += NW) {
            double w = 0.0;
            for (int i = kk + lane; i < sp; i += 64)
                w += (i == kk ? 1.0 : hh[i * SK_SMAX + kk]) * sA[l * LA + i];
            w = wave_sum(w) * tau;
            for (int i = kk + lane; i < sp; i += 64)
                sA[l * LA + i] -= w * (i == kk ? 1.0 : hh[i * SK_SMAX + kk]);
        }
        __syncthreads();
    }
    for (int e = tid; e < sp * k; e += SK_SVD_TH) {
        const int a = e / k, l = e % k;
        Lm[a * SK_CAP_MAX + l] = sA[l * LA + a];
    }
}

// the bases: alpha's rows U = (A X) R, beta's rows V = (A^T Y) L, into the
// panel columns col0 .. col0 + k - 1 (64 rows per work-group, the rows'
// sketch entries staged in LDS, wave w taking columns w, w + 4, ...)
__global__ __launch_bounds__(256) void sk_form_kernel(SketchArgs S)
{
    const Chunk ch = S.chunks[blockIdx.x];
    const int64_t h = ch.node;
    int64_t lo, mid, hi;
    int s, sp;
    sk_sizes(S, h, lo, mid, hi, s, sp);
    const int k = S.rank[h];
    if (s == 0 || k == 0)
        return;   // the whole work-group
    __shared__ double sS[SK_ROWS][SK_SPMAX + 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nsamp = ch.side ? sp : s;
    const int64_t n = S.n;
    for (int e = tid; e < SK_ROWS * nsamp; e += 256) {
        const int j = e / SK_ROWS, i = e % SK_ROWS;
        const int64_t row = ch.lo + i;
        sS[i][j] = row < ch.hi ? S.sk[(int64_t)j * n + row] : 0.0;
    }
    __syncthreads();
    const int64_t loc = h - S.node0;
    const double *M = S.fac + loc * SK_FAC + (ch.side ? SK_SMAX * SK_CAP_MAX : 0);
    const int64_t row = ch.lo + lane;
    for (int l = wid; l < k; l += 4) {
        double v = 0.0;
        for (int j = 0; j < nsamp; ++j)
            v += sS[lane][j] * M[j * SK_CAP_MAX + l];
        if (row < ch.hi)
            S.W[(S.col0 + l) * n + row] = v;
    }
}

// Compress every level's blocks into the W panels and write rank[] and
// status[] per node (the caller zeroed them and reads the statistics).
void run_sketch_levels(Pipeline &P, int *rank, int *status)
{
    const Plan &p = *P.plan;
    if (p.cap > SK_CAP_MAX)
        throw Error{HODLR_EINVAL, "the sketch compressor needs max_rank <= 64"};
    SketchArgs S;
    S.kp = P.kp;
    S.x = P.x;
    S.n = p.n;
    S.start = p.d_start;
    S.end = p.d_end;
    S.cap = p.cap;
    S.tol = P.tol;
    S.sk = wsp<double>(P, P.lay.sk_buf);
    S.part = wsp<double>(P, P.lay.sk_part);
    S.core = wsp<double>(P, P.lay.sk_core);
    S.fac = wsp<double>(P, P.lay.sk_fac);
    S.rank = rank;
    S.status = status;
    S.W = wsp<double>(P, P.lay.W);
    for (int d = 0; d < p.L; ++d) {
        const unsigned nch = (unsigned)p.sk[d].size();
        const unsigned nodes = (unsigned)(p.first_at(d + 1) - p.first_at(d));
        S.chunks = p.d_sk[d];
        S.abase = p.d_sk_abase[d];
        S.acnt = p.d_sk_acnt[d];
        S.node0 = p.first_at(d);
        S.col0 = p.cofa[d + 1];
        // the widest sketch of the level (tiles of 16 sketch columns)
        int wmax = 0;
        for (int64_t hh = p.first_at(d); hh < p.first_at(d + 1); ++hh) {
            const int64_t a = (p.end[hh] - p.start[hh]) / 2, b = p.end[hh] - p.start[hh] - a;
            const int64_t t = std::min<int64_t>({(int64_t)p.cap + SK_OVER_X, a, b});
            if (t > 0)
                wmax = std::max<int>(wmax, (int)std::min<int64_t>(t + SK_OVER_Y, a));
            wmax = std::max<int>(wmax, (int)std::max<int64_t>(t, 0));
        }
        if (nch == 0 || wmax == 0) {
            // no block to compress: ranks 0
            sk_svd_kernel<<<nodes, SK_SVD_TH, 0, P.stream>>>(S);
            HIP_TRY(hipGetLastError());
            continue;
        }
        {
            ProfScope ps(P.stream, PS_SKETCH);
            const int nt = (wmax + 15) / 16;
            switch (nt) {
            case 1: sketch_kernel<1><<<nch, 256, 0, P.stream>>>(S); break;
            case 2: sketch_kernel<2><<<nch, 256, 0, P.stream>>>(S); break;
            case 3: sketch_kernel<3><<<nch, 256, 0, P.stream>>>(S); break;
            case 4: sketch_kernel<4><<<nch, 256, 0, P.stream>>>(S); break;
            case 5: sketch_kernel<5><<<nch, 256, 0, P.stream>>>(S); break;
            default: sketch_kernel<6><<<nch, 256, 0, P.stream>>>(S); break;
            }
            HIP_TRY(hipGetLastError());
        }
        {
            ProfScope ps(P.stream, PS_SKETCH_CORE);
            sk_core_sum_kernel<<<dim3(nodes, (unsigned)((SK_CORE + 255) / 256)), 256, 0, P.stream>>>(S);
            sk_svd_kernel<<<nodes, SK_SVD_TH, 0, P.stream>>>(S);
            sk_form_kernel<<<nch, 256, 0, P.stream>>>(S);
            HIP_TRY(hipGetLastError());
        }
    }
}

}  // namespace hodlr
