// Projected level stage for a likelihood (log det C and C^{-1} y).
//
// The factorization of §3.2 applies the block-diagonal inverses to every
// ancestor basis at every level, which moves O(n r L^2) bytes.  The
// likelihood needs those applied bases only through their projections onto
// the bases themselves: for a node tau let Z_tau hold, on tau's rows, the
// right-hand side y and the bases of tau's ancestors and of tau itself (the
// used columns of depths 1..depth(tau)), and let G_tau = Z_tau^T K_tau^{-1} Z_tau,
// where K_tau is tau's diagonal block of the HODLR matrix.  With children
// alpha, beta and D the columns of depth(tau)+1 (W_alpha, W_beta),
// K_tau = diag(K_alpha, K_beta)(I + diag(K_alpha^{-1} W_alpha, K_beta^{-1} W_beta)
// [[0, W_beta^T], [W_alpha^T, 0]]) (§3.2's low-rank update of the identity), and
// by Sylvester's determinant theorem and Sherman-Morrison-Woodbury:
//
//   M_tau = [[I, P], [Q, I]],  P = G_beta[D, D],  Q = G_alpha[D, D],
//   det M_tau = det N,  N = I - Q P                       (§4)
//   S = M_tau^{-1} [G_beta[D, A]; G_alpha[D, A]]  (A: tau's own columns)
//     = [R1 - P S2; S2],  S2 = N^{-1}(R2 - Q R1),  R1 = G_beta[D, A], R2 = G_alpha[D, A]
//   G_tau = G_alpha[A, A] + G_beta[A, A] - G_alpha[A, D] S1 - G_beta[A, D] S2
//
// At a leaf G_lambda = Z^T (C_lambda^{-1} Z) from the leaf factor's applied
// panel; at the root G = y^T C^{-1} y.  The same recursion run downwards gives
// C^{-1} y: on tau's rows K_tau^{-1} Z_tau c = K_alpha^{-1} Z_alpha [c; -S1 c]
// (and [c; -S2 c] on beta's rows), so each leaf's coefficients come from the
// S of its ancestors and z = (C_lambda^{-1} Z_lambda) c_lambda.  The coupling
// matrices and determinants are those of the level-by-level factorization;
// only the O(n r L^2) panel traffic is gone (G and S are O(n r^2 / leaf)).
#include "common.h"

namespace hodlr {

namespace {

constexpr int PJ_RC = 16;   // rows per LDS chunk of the leaf projection

struct ProjArgs {
    int64_t n = 0;
    const double *W = nullptr;   // bases panel (column-major n x ncol)
    const char *Xt = nullptr;    // applied panel after the leaf factor (PT)
    const double *y = nullptr;   // right-hand side in tree order
    const int *cols = nullptr;   // used columns, compact order, cols[0] = 0
    const int64_t *start = nullptr, *end = nullptr;   // per heap node
    double *Gin = nullptr, *Gout = nullptr;   // children's and this level's G store
    double *S = nullptr;                      // this level's S store (2w x m per node)
    double *node_ld = nullptr;
    int *status = nullptr;
    int64_t node0 = 0;   // heap index of the level's first node
    int m = 0, w = 0;    // columns of this level's G (cnt[d]); width of depth d+1
    BatchArgs B;
};

// G_lambda = Z_lambda^T Xt_lambda over one leaf's rows (16 x 16 threads, each an
// MB x MB block of the at most 16 MB x 16 MB result); column 0 of Z is y.
template <typename PT, int MB>
__global__ __launch_bounds__(256) void proj_leaf_kernel(ProjArgs A)
{
    const int it = blockIdx.z;
    const int64_t h = A.node0 + blockIdx.x;
    const int64_t s = A.start[h], e = A.end[h];
    const int64_t n = A.n;
    const double *W = ioff(A.W, A.B, it);
    const PT *X = (const PT *)ioff(A.Xt, A.B, it);
    const double *y = A.y + it * A.B.ystride;
    const int m = A.m;
    __shared__ double zs[PJ_RC][16 * MB + 1], xs[PJ_RC][16 * MB + 1];
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    double acc[MB][MB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < MB; ++b)
            acc[a][b] = 0.0;
    for (int64_t r0 = s; r0 < e; r0 += PJ_RC) {
        for (int idx = tid; idx < PJ_RC * m; idx += 256) {
            const int rr = idx % PJ_RC, k = idx / PJ_RC;
            const int64_t row = r0 + rr;
            const int64_t rc = row < e ? row : e - 1;   // clamped: loads never wait on a branch
            const int64_t c = A.cols[k];
            const double *zp = k == 0 ? y : W + c * n;
            double zv = zp[rc];
            double xv = (double)X[c * n + rc];
            asm volatile("" : "+v"(zv), "+v"(xv));
            zs[rr][k] = row < e ? zv : 0.0;
            xs[rr][k] = row < e ? xv : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < PJ_RC; ++rr) {
            double za[MB], xb[MB];
#pragma unroll
            for (int a = 0; a < MB; ++a)
                za[a] = zs[rr][ty + 16 * a];
#pragma unroll
            for (int b = 0; b < MB; ++b)
                xb[b] = xs[rr][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < MB; ++a)
#pragma unroll
                for (int b = 0; b < MB; ++b)
                    acc[a][b] = fma(za[a], xb[b], acc[a][b]);
        }
        __syncthreads();
    }
    double *G = ioff(A.Gout, A.B, it) + (int64_t)blockIdx.x * m * m;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            const int i = ty + 16 * a, j = tx + 16 * b;
            if (i < m && j < m)
                G[(int64_t)i * m + j] = acc[a][b];
        }
}

typedef double d4 __attribute__((ext_vector_type(4)));

// The same product on FP64 MFMA for at most 16 TM <= 64 columns, one wave per
// leaf.  Chunks of 16 rows go through LDS: each column's 16 rows are one
// coalesced 128-byte load (the next chunk's loads are issued before this
// chunk's products), and lane (r, q) takes row 4 u + q of column 16 T + r of
// Z and of Xt from LDS as the A and B operands of the 16 x 16 x 4 product;
// tile (T, U) accumulates G[16 T + q + 4 t][16 U + r] in element t.
constexpr int PJ_MLD = 65;   // LDS row length of the staged chunks
template <typename PT, int TM>
__global__ __launch_bounds__(64) void proj_leaf_mfma_kernel(ProjArgs A)
{
    constexpr int NV = (16 * 16 * TM + 63) / 64;   // staged values per lane and operand
    const int it = blockIdx.z;
    const int64_t h = A.node0 + blockIdx.x;
    const int64_t s = A.start[h], e = A.end[h];
    const int64_t n = A.n;
    const double *W = ioff(A.W, A.B, it);
    const PT *X = (const PT *)ioff(A.Xt, A.B, it);
    const double *y = A.y + it * A.B.ystride;
    const int m = A.m;
    const int l = threadIdx.x, r = l & 15, q = l >> 4;
    __shared__ double zs[16 * PJ_MLD], xs[16 * PJ_MLD];
    // the staged values of this lane: row r of columns k = q + 4 j (value
    // l + 64 j of the chunk); columns past m read column 0 and are zeroed, and
    // Z's column 0 (lane q = 0, j = 0) is y
    int64_t off[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int k = q + 4 * j;
        off[j] = (int64_t)A.cols[k < m ? k : 0] * n;
    }
    const double *z0 = q == 0 ? y : W + off[0];
    double zv[NV], xv[NV];
    auto load = [&](int64_t r0) {
        const int64_t row = r0 + r;
        const int64_t rc = row < e ? row : e - 1;   // clamped: loads never wait on a branch
        zv[0] = z0[rc];
        xv[0] = (double)X[off[0] + rc];
#pragma unroll
        for (int j = 1; j < NV; ++j) {
            zv[j] = W[off[j] + rc];
            xv[j] = (double)X[off[j] + rc];
        }
    };
    d4 acc[TM][TM];
#pragma unroll
    for (int T = 0; T < TM; ++T)
#pragma unroll
        for (int U = 0; U < TM; ++U)
            acc[T][U] = d4{0.0, 0.0, 0.0, 0.0};
    if (s < e)
        load(s);
    for (int64_t r0 = s; r0 < e; r0 += 16) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int k = q + 4 * j;
            asm volatile("" : "+v"(zv[j]), "+v"(xv[j]));
            const bool in = k < m && r0 + r < e;
            zs[r * PJ_MLD + k] = in ? zv[j] : 0.0;
            xs[r * PJ_MLD + k] = in ? xv[j] : 0.0;
        }
        __syncthreads();
        if (r0 + 16 < e)
            load(r0 + 16);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double za[TM], xb[TM];
#pragma unroll
            for (int T = 0; T < TM; ++T) {
                za[T] = zs[(4 * u + q) * PJ_MLD + 16 * T + r];
                xb[T] = xs[(4 * u + q) * PJ_MLD + 16 * T + r];
            }
#pragma unroll
            for (int T = 0; T < TM; ++T)
#pragma unroll
                for (int U = 0; U < TM; ++U)
                    acc[T][U] = __builtin_amdgcn_mfma_f64_16x16x4f64(za[T], xb[U], acc[T][U],
                                                                     0, 0, 0);
        }
        __syncthreads();
    }
    double *G = ioff(A.Gout, A.B, it) + (int64_t)blockIdx.x * m * m;
#pragma unroll
    for (int T = 0; T < TM; ++T)
#pragma unroll
        for (int U = 0; U < TM; ++U)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = 16 * T + q + 4 * t, j = 16 * U + r;
                if (i < m && j < m)
                    G[(int64_t)i * m + j] = acc[T][U][t];
            }
}

// One level upwards: one wave per node of depth d (see the file comment).
// Dynamic LDS: P, Q, N (w x w), R1/S1 and R2/S2 (w x m), G_alpha[A, D] and
// G_beta[A, D] (m x w).
__global__ __launch_bounds__(64) void proj_up_kernel(ProjArgs A)
{
    const int it = blockIdx.z;
    const int i = blockIdx.x;
    const int m = A.m, w = A.w, mc = m + w;
    const int lane = threadIdx.x;
    const double *Ga = ioff(A.Gin, A.B, it) + (int64_t)(2 * i) * mc * mc;
    const double *Gb = Ga + (int64_t)mc * mc;
    double *Go = ioff(A.Gout, A.B, it) + (int64_t)i * m * m;
    extern __shared__ double sh[];
    double *sP = sh, *sQ = sP + w * w, *sN = sQ + w * w;
    double *s1 = sN + w * w, *s2 = s1 + w * m;
    double *ad = s2 + w * m, *bd = ad + m * w;
    __shared__ int piv;
    __shared__ int bad;
    if (lane == 0)
        bad = 0;
    for (int idx = lane; idx < w * w; idx += 64) {
        const int r = idx / w, c = idx % w;
        sP[idx] = Gb[(int64_t)(m + r) * mc + m + c];
        sQ[idx] = Ga[(int64_t)(m + r) * mc + m + c];
    }
    for (int idx = lane; idx < w * m; idx += 64) {
        const int r = idx / m, c = idx % m;
        s1[idx] = Gb[(int64_t)(m + r) * mc + c];
        s2[idx] = Ga[(int64_t)(m + r) * mc + c];
        const int a = idx / w, k = idx % w;   // the same count, m x w
        ad[idx] = Ga[(int64_t)a * mc + m + k];
        bd[idx] = Gb[(int64_t)a * mc + m + k];
    }
    __syncthreads();
    // N = I - Q P; T = R2 - Q R1 (in place of R2)
    for (int idx = lane; idx < w * w; idx += 64) {
        const int r = idx / w, c = idx % w;
        double v = r == c ? 1.0 : 0.0;
        for (int k = 0; k < w; ++k)
            v -= sQ[r * w + k] * sP[k * w + c];
        sN[idx] = v;
    }
    for (int idx = lane; idx < w * m; idx += 64) {
        const int r = idx / m, c = idx % m;
        double v = s2[idx];
        for (int k = 0; k < w; ++k)
            v -= sQ[r * w + k] * s1[k * m + c];
        s2[idx] = v;
    }
    __syncthreads();
    // N S2 = T by elimination with partial pivoting; log det N from the pivots
    double lg = 0.0;
    int flips = 0;
    for (int k = 0; k < w; ++k) {
        if (lane == 0) {
            int p = k;
            double best = fabs(sN[k * w + k]);
            for (int r = k + 1; r < w; ++r)
                if (fabs(sN[r * w + k]) > best) {
                    best = fabs(sN[r * w + k]);
                    p = r;
                }
            piv = p;
            if (!(best > 0.0))
                bad = 1;
        }
        __syncthreads();
        const int p = piv;
        if (p != k) {
            for (int c = lane; c < w; c += 64) {
                const double t = sN[k * w + c];
                sN[k * w + c] = sN[p * w + c];
                sN[p * w + c] = t;
            }
            for (int c = lane; c < m; c += 64) {
                const double t = s2[k * m + c];
                s2[k * m + c] = s2[p * m + c];
                s2[p * m + c] = t;
            }
            ++flips;
        }
        __syncthreads();
        const double pv = sN[k * w + k];
        lg += log(fabs(pv));
        flips += pv < 0.0 ? 1 : 0;
        const double rp = bad ? 0.0 : 1.0 / pv;
        for (int r = k + 1; r < w; ++r) {
            const double f = sN[r * w + k] * rp;
            for (int c = k + 1 + lane; c < w; c += 64)
                sN[r * w + c] -= f * sN[k * w + c];
            for (int c = lane; c < m; c += 64)
                s2[r * m + c] -= f * s2[k * m + c];
        }
        __syncthreads();
    }
    for (int k = w - 1; k >= 0; --k) {
        const double rp = bad ? 0.0 : 1.0 / sN[k * w + k];
        for (int c = lane; c < m; c += 64) {
            double v = s2[k * m + c];
            for (int j = k + 1; j < w; ++j)
                v -= sN[k * w + j] * s2[j * m + c];
            s2[k * m + c] = v * rp;
        }
        __syncthreads();
    }
    // S1 = R1 - P S2
    for (int idx = lane; idx < w * m; idx += 64) {
        const int r = idx / m, c = idx % m;
        double v = s1[idx];
        for (int k = 0; k < w; ++k)
            v -= sP[r * w + k] * s2[k * m + c];
        s1[idx] = v;
    }
    __syncthreads();
    double *S = ioff(A.S, A.B, it) + (int64_t)i * 2 * w * m;
    for (int idx = lane; idx < w * m; idx += 64) {
        S[idx] = s1[idx];
        S[w * m + idx] = s2[idx];
    }
    // four outputs per lane at a time, their eight loads issued first
    // (clamped indices, stores masked)
    const int mm = m * m;
    for (int idx0 = lane; idx0 < mm; idx0 += 256) {
        double v[4];
        int ix[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ix[u] = min(idx0 + 64 * u, mm - 1);
            const int a = ix[u] / m, b = ix[u] % m;
            v[u] = Ga[(int64_t)a * mc + b] + Gb[(int64_t)a * mc + b];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int a = ix[u] / m, b = ix[u] % m;
            for (int k = 0; k < w; ++k)
                v[u] -= ad[a * w + k] * s1[k * m + b] + bd[a * w + k] * s2[k * m + b];
            if (idx0 + 64 * u < mm)
                Go[idx0 + 64 * u] = v[u];
        }
    }
    if (lane == 0) {
        double *ld = ioff(A.node_ld, A.B, it);
        if (bad || (flips & 1)) {
            atomicOr(ioff(A.status, A.B, it), DS_NOTSPD_NODE);
            lg = __builtin_nan("");
        }
        ld[A.node0 + i] = lg;
    }
}

struct ProjDown {
    int64_t soff[HODLR_MAX_LEVELS];   // per level d: first double of its S store
    int m[HODLR_MAX_LEVELS + 1];      // cnt[d]
    int w[HODLR_MAX_LEVELS + 1];      // rmax[d]
    int L = 0;
};

// Downwards: one wave per leaf walks its ancestors from the root, building
// the leaf's coefficients c (the ancestors' -S c pieces), then writes
// z = Xt_lambda c into column 0 of the applied panel on the leaf's rows.
template <typename PT>
__global__ __launch_bounds__(64) void proj_down_kernel(ProjArgs A, ProjDown D)
{
    const int it = blockIdx.z;
    const int64_t lam = blockIdx.x;
    const int L = D.L, lane = threadIdx.x;
    __shared__ double c[PJ_MMAX];
    if (lane == 0)
        c[0] = 1.0;
    const double *S0 = ioff(A.S, A.B, it);
    for (int d = 0; d < L; ++d) {
        const int64_t i = lam >> (L - d);
        const int side = (int)((lam >> (L - d - 1)) & 1);
        const int m = D.m[d], w = D.w[d + 1];
        const double *S = S0 + D.soff[d] + i * 2 * w * m + (int64_t)side * w * m;
        __syncthreads();
        double v = 0.0;
        if (lane < w)
            for (int j = 0; j < m; ++j)
                v += S[(int64_t)lane * m + j] * c[j];
        __syncthreads();
        if (lane < w)
            c[m + lane] = -v;
    }
    __syncthreads();
    const int mL = D.m[L];
    const int64_t h = (((int64_t)1) << L) - 1 + lam;
    const int64_t s = A.start[h], e = A.end[h], n = A.n;
    PT *X = (PT *)ioff(A.Xt, A.B, it);
    for (int64_t row = s + lane; row < e; row += 64) {
        double z = 0.0;
        for (int k = 0; k < mL; ++k)
            z += (double)X[(int64_t)A.cols[k] * n + row] * c[k];
        X[row] = (PT)z;
    }
}

template <typename PT>
void leaf_launch(int mb, dim3 g, hipStream_t s, const ProjArgs &A)
{
    switch (mb) {
    case 1: proj_leaf_mfma_kernel<PT, 1><<<g, 64, 0, s>>>(A); return;
    case 2: proj_leaf_mfma_kernel<PT, 2><<<g, 64, 0, s>>>(A); return;
    case 3: proj_leaf_mfma_kernel<PT, 3><<<g, 64, 0, s>>>(A); return;
    case 4: proj_leaf_mfma_kernel<PT, 4><<<g, 64, 0, s>>>(A); return;
    default: break;
    }
    switch (mb) {
    case 1: proj_leaf_kernel<PT, 1><<<g, 256, 0, s>>>(A); break;
    case 2: proj_leaf_kernel<PT, 2><<<g, 256, 0, s>>>(A); break;
    case 3: proj_leaf_kernel<PT, 3><<<g, 256, 0, s>>>(A); break;
    case 4: proj_leaf_kernel<PT, 4><<<g, 256, 0, s>>>(A); break;
    case 5: proj_leaf_kernel<PT, 5><<<g, 256, 0, s>>>(A); break;
    case 6: proj_leaf_kernel<PT, 6><<<g, 256, 0, s>>>(A); break;
    case 7: proj_leaf_kernel<PT, 7><<<g, 256, 0, s>>>(A); break;
    default: proj_leaf_kernel<PT, 8><<<g, 256, 0, s>>>(A); break;
    }
}

size_t up_lds(int m, int w) { return sizeof(double) * (3 * (size_t)w * w + 4 * (size_t)w * m); }

// doubles of the G store of depth j, and of all levels' S stores
int64_t g_doubles(const Pipeline &P, int j)
{
    return ((int64_t)1 << j) * (int64_t)P.cnt[j] * P.cnt[j];
}

}  // namespace

bool proj_fits(const Pipeline &P)
{
    const Plan &p = *P.plan;
    if (!P.rhs || P.lay.store_leaf || p.L < 1 || p.L >= HODLR_MAX_LEVELS ||
        p.level_form != 0 || P.cnt[p.L] > PJ_MMAX)
        return false;
    const int64_t tb = (int64_t)((P.lay.Sbuf - P.lay.Tbuf) / sizeof(double));
    const int64_t sb = (int64_t)((P.lay.small - P.lay.Sbuf) / sizeof(double));
    int64_t st = 0;
    for (int j = p.L; j >= 0; --j) {
        if (g_doubles(P, j) > ((p.L - j) % 2 == 0 ? tb : sb))
            return false;
        if (j < p.L) {
            const int w = P.rmax[j + 1];
            if (w > PJ_WMAX || up_lds(P.cnt[j], w) > 60 * 1024)
                return false;
            st += ((int64_t)1 << j) * 2 * w * P.cnt[j];
        }
    }
    return st <= P.lay.lvl_part_cap;
}

void run_levels_projected(Pipeline &P)
{
    const Plan &p = *P.plan;
    const int L = p.L;
    ProjArgs A;
    A.n = p.n;
    A.W = wsp<double>(P, P.lay.W);
    A.Xt = P.ws + P.lay.Xt;
    A.y = P.rhs;
    A.cols = wsp<int>(P, P.lay.cols);
    A.start = p.d_start;
    A.end = p.d_end;
    A.node_ld = wsp<double>(P, P.lay.node_ld);
    A.status = wsp<int>(P, P.lay.status);
    A.B = P.batch;
    double *gbuf[2] = {wsp<double>(P, P.lay.Tbuf), wsp<double>(P, P.lay.Sbuf)};
    double *sstore = wsp<double>(P, P.lay.lvl_part);
    ProjDown D;
    D.L = L;
    int64_t so = 0;
    for (int d = 0; d < L; ++d) {
        D.soff[d] = so;
        so += ((int64_t)1 << d) * 2 * P.rmax[d + 1] * P.cnt[d];
    }
    for (int d = 0; d <= L; ++d) {
        D.m[d] = P.cnt[d];
        D.w[d] = d >= 1 ? P.rmax[d] : 0;
    }
    {
        ProfScope ps(P.stream, PS_LVL_REDUCE);
        A.node0 = p.first_at(L);
        A.m = P.cnt[L];
        A.Gout = gbuf[0];
        const int mb = (A.m + 15) / 16;
        const dim3 g((unsigned)p.nleaf, 1, P.nitems);
        if (p.f32())
            leaf_launch<float>(mb, g, P.stream, A);
        else
            leaf_launch<double>(mb, g, P.stream, A);
        HIP_TRY(hipGetLastError());
    }
    {
        ProfScope ps(P.stream, PS_LVL_SOLVE);
        for (int d = L - 1; d >= 0; --d) {
            A.node0 = p.first_at(d);
            A.m = P.cnt[d];
            A.w = P.rmax[d + 1];
            A.Gin = gbuf[(L - d - 1) % 2];
            A.Gout = gbuf[(L - d) % 2];
            A.S = sstore + D.soff[d];
            const dim3 g((unsigned)(p.first_at(d + 1) - p.first_at(d)), 1, P.nitems);
            proj_up_kernel<<<g, 64, up_lds(A.m, A.w), P.stream>>>(A);
            HIP_TRY(hipGetLastError());
        }
    }
    {
        ProfScope ps(P.stream, PS_LVL_UPDATE);
        A.S = sstore;
        const dim3 g((unsigned)p.nleaf, 1, P.nitems);
        if (p.f32())
            proj_down_kernel<float><<<g, 64, 0, P.stream>>>(A, D);
        else
            proj_down_kernel<double><<<g, 64, 0, P.stream>>>(A, D);
        HIP_TRY(hipGetLastError());
    }
}

}  // namespace hodlr
