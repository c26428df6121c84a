// Batched adaptive cross approximation (ACA) of every off-diagonal block
// K(alpha, beta) of the tree, all levels at once (§3.1 of the paper: an
// approximate partially pivoted LU that builds A ~ sum_k u_k v_k^T from rows
// and columns of A, with a sub-sampled error estimate).
//
// Each ACA step is two launches over all blocks still active:
//   row pass    -- residual row v = A(i*, :) - sum_l u_l(i*) v_l over beta,
//                  written as column k of the beta rows of the depth-(d+1)
//                  panel; the last work-group of a block picks the pivot
//                  column j* (first max |v|) and records v.v_l;
//   column pass -- u = (A(:, j*) - sum_l v_l(j*) u_l) / v(j*) over alpha,
//                  written as column k of the alpha rows; the last
//                  work-group updates ||S_k||_F^2, applies the stopping test
//                  ||u|| ||v|| <= tol ||S_k||_F and picks the next pivot row
//                  (first max |u| over unused rows).
// A zero pivot marks the row used and retries the unused row nearest the
// split; the first row is the one next to the split.  Entries are evaluated
// on the fly from the ordered coordinates; a work-group handles ACA_CHUNK
// consecutive indices, so the coordinate and panel accesses are coalesced.
#include "common.h"

namespace hodlr {

struct AcaArgs {
    const double *x;
    int64_t n;
    KParams kp;
    double tol;
    double *W;
    const int64_t *start, *end;
    const int64_t *cofa;   // device copy of column offsets per depth
    AcaState *st;
    int *used;
    double *vdots;
    int vstride;
    double *part;
    int pw;
    int *cnt;
    int *active;
    const Chunk *chunks;
    const int *nch;
    const int *base;
};

__device__ __forceinline__ int depth_of_node(int64_t h)
{
    return 63 - __clzll((unsigned long long)(h + 1));
}

__global__ void aca_init_kernel(AcaArgs A, int64_t nint, int cap)
{
    int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (h >= nint)
        return;
    int64_t s = A.start[h], e = A.end[h], m = s + (e - s) / 2;
    int64_t na = m - s, nb = e - m;
    int64_t full = na < nb ? na : nb;
    int c = (int)(cap < full ? cap : full);
    AcaState t;
    t.k = 0;
    t.istar = (int)(na - 1);
    t.jstar = 0;
    t.done = (c <= 0) ? ACA_EXHAUSTED : ACA_ACTIVE;
    t.phase = PH_ROW;
    t.zeros = 0;
    t.nused = 0;
    t.cap = c;
    t.usercap = (cap < full) ? 1 : 0;
    t.pad_ = 0;
    t.delta = 0.0;
    t.v2 = 0.0;
    t.s2 = 0.0;
    A.st[h] = t;
    A.cnt[h] = 0;
    if (t.done == ACA_ACTIVE)
        atomicAdd(A.active, 1);
}

// block-wide reductions over 256 threads (4 waves)
struct BlockRed {
    double v[4];
    int64_t i[4];
};

template <bool ROW>
__global__ __launch_bounds__(ACA_THREADS) void aca_pass_kernel(AcaArgs A)
{
    const Chunk ch = A.chunks[blockIdx.x];
    const int h = ch.node;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    __shared__ AcaState sst;
    __shared__ double sfix[RMAX_ABS];        // u_l(i*) (row pass) or v_l(j*) (column pass)
    __shared__ int sused[USED_MAX];
    __shared__ double sdot[4][RMAX_ABS + 1];
    __shared__ BlockRed sred;
    __shared__ double ssgn[4];
    __shared__ int s_last;
    if (tid == 0)
        sst = A.st[h];
    __syncthreads();
    if (sst.done != ACA_ACTIVE || sst.phase != (ROW ? PH_ROW : PH_COL))
        return;
    const int k = sst.k;
    const int64_t s = A.start[h], e = A.end[h], m = s + (e - s) / 2;
    const int64_t n = A.n;
    const int64_t col0 = A.cofa[depth_of_node(h) + 1];
    double *__restrict__ W = A.W;
    // the fixed index this pass crosses: pivot row (row pass) or pivot column
    const int64_t fix = ROW ? (s + sst.istar) : (m + sst.jstar);
    for (int l = tid; l < k; l += ACA_THREADS)
        sfix[l] = W[(col0 + l) * n + fix];
    if (!ROW)
        for (int t = tid; t < sst.nused; t += ACA_THREADS)
            sused[t] = A.used[(int64_t)h * USED_MAX + t];
    __syncthreads();
    const double delta = sst.delta;
    double val[ACA_EPT];
    double bestv = -1.0, bests = 0.0;
    int64_t besti = INT64_MAX;
    double sq = 0.0;
#pragma unroll
    for (int t = 0; t < ACA_EPT; ++t) {
        int64_t g = ch.lo + tid + (int64_t)t * ACA_THREADS;
        val[t] = 0.0;
        if (g < ch.hi) {
            double a = kentry(A.kp, A.x, n, ROW ? fix : g, ROW ? g : fix);
            for (int l = 0; l < k; ++l)
                a -= sfix[l] * W[(col0 + l) * n + g];
            if (!ROW)
                a = a / delta;
            W[(col0 + k) * n + g] = a;
            val[t] = a;
            sq += a * a;
            bool eligible = true;
            if (!ROW) {
                int li = (int)(g - s);
                for (int q = 0; q < sst.nused; ++q)
                    eligible = eligible && (sused[q] != li);
            }
            double av = fabs(a);
            if (eligible && av > bestv) {
                bestv = av;
                bests = a;
                besti = g;
            }
        }
    }
    // dots with the earlier terms of the same side
    for (int l = 0; l < k; ++l) {
        double dsum = 0.0;
#pragma unroll
        for (int t = 0; t < ACA_EPT; ++t) {
            int64_t g = ch.lo + tid + (int64_t)t * ACA_THREADS;
            if (g < ch.hi)
                dsum += val[t] * W[(col0 + l) * n + g];
        }
        dsum = wave_sum(dsum);
        if (lane == 0)
            sdot[wid][l] = dsum;
    }
    sq = wave_sum(sq);
    if (lane == 0)
        sdot[wid][k] = sq;
    wave_argmax_signed(bestv, besti, bests);
    if (lane == 0) {
        sred.v[wid] = bestv;
        sred.i[wid] = besti;
        ssgn[wid] = bests;
    }
    __syncthreads();
    double *rec = A.part + (int64_t)ch.part * A.pw;
    if (tid == 0) {
        double bv = sred.v[0], bs = ssgn[0];
        int64_t bi = sred.i[0];
        for (int w = 1; w < 4; ++w)
            if (sred.v[w] > bv || (sred.v[w] == bv && sred.i[w] < bi)) {
                bv = sred.v[w];
                bi = sred.i[w];
                bs = ssgn[w];
            }
        rec[0] = bv;
        rec[1] = (bi == INT64_MAX) ? -1.0 : (double)bi;
        rec[2] = sdot[0][k] + sdot[1][k] + sdot[2][k] + sdot[3][k];
        rec[3] = bs;
    }
    for (int l = tid; l < k; l += ACA_THREADS)
        rec[4 + l] = sdot[0][l] + sdot[1][l] + sdot[2][l] + sdot[3][l];
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        int prev = atomicAdd(&A.cnt[h], 1);
        s_last = (prev == A.nch[h] - 1);
    }
    __syncthreads();
    if (!s_last)
        return;
    __threadfence();
    // ---- the last work-group of this block combines the partial records
    const int nch = A.nch[h];
    const double *prt = A.part + (int64_t)A.base[h] * A.pw;
    // dots (l < k) and the squared norm (slot k), one accumulator per thread
    for (int l = tid; l <= k; l += ACA_THREADS) {
        double acc = 0.0;
        int slot = (l < k) ? 4 + l : 2;
        for (int c = 0; c < nch; ++c)
            acc += ld_coherent(prt + (int64_t)c * A.pw + slot);
        sdot[0][l] = acc;
    }
    double bv = -1.0, sv = 0.0;
    int64_t bi = INT64_MAX;
    for (int c = tid; c < nch; c += ACA_THREADS) {
        double v = ld_coherent(prt + (int64_t)c * A.pw + 0);
        double di = ld_coherent(prt + (int64_t)c * A.pw + 1);
        int64_t i = di < 0.0 ? INT64_MAX : (int64_t)di;
        if (v > bv || (v == bv && i < bi)) {
            bv = v;
            bi = i;
            sv = ld_coherent(prt + (int64_t)c * A.pw + 3);
        }
    }
    wave_argmax_signed(bv, bi, sv);
    __syncthreads();   // stage-1 readers of sred/ssgn are done
    if (lane == 0) {
        sred.v[wid] = bv;
        sred.i[wid] = bi;
        ssgn[wid] = sv;
    }
    __syncthreads();
    if (tid != 0)
        return;
    bv = sred.v[0];
    bi = sred.i[0];
    sv = ssgn[0];
    for (int w = 1; w < 4; ++w)
        if (sred.v[w] > bv || (sred.v[w] == bv && sred.i[w] < bi)) {
            bv = sred.v[w];
            bi = sred.i[w];
            sv = ssgn[w];
        }
    AcaState t = sst;
    const int64_t na = m - s;
    int *used = A.used + (int64_t)h * USED_MAX;
    if (ROW) {
        if (t.nused < USED_MAX)
            used[t.nused] = t.istar;
        t.nused += 1;
        if (bv == 0.0) {
            t.zeros += 1;
            if (t.zeros > ZERO_RETRY || t.nused >= na || t.nused >= USED_MAX) {
                t.done = ACA_EXHAUSTED;
            } else {
                // unused row nearest the split
                int cand = (int)na - 1;
                for (; cand >= 0; --cand) {
                    bool u = false;
                    for (int q = 0; q < t.nused; ++q)
                        u = u || (used[q] == cand);
                    if (!u)
                        break;
                }
                t.istar = cand;
            }
        } else {
            t.zeros = 0;
            t.jstar = (int)(bi - m);
            t.delta = sv;
            t.v2 = sdot[0][k];
            for (int l = 0; l < k; ++l)
                A.vdots[(int64_t)h * A.vstride + l] = sdot[0][l];
            t.phase = PH_COL;
        }
    } else {
        double u2 = sdot[0][k];
        double cross = 0.0;
        for (int l = 0; l < k; ++l)
            cross += sdot[0][l] * A.vdots[(int64_t)h * A.vstride + l];
        t.s2 += u2 * t.v2 + 2.0 * cross;
        t.k = k + 1;
        double s2 = t.s2 > 0.0 ? t.s2 : 0.0;
        if (sqrt(u2) * sqrt(t.v2) <= A.tol * sqrt(s2)) {
            t.done = ACA_CONVERGED;
        } else if (t.k >= t.cap) {
            t.done = t.usercap ? ACA_CAPPED : ACA_CONVERGED;
        } else if (t.nused >= na || t.nused >= USED_MAX || bv < 0.0) {
            t.done = ACA_EXHAUSTED;
        } else {
            t.istar = (int)(bi - s);
            t.phase = PH_ROW;
        }
    }
    if (t.done != ACA_ACTIVE)
        atomicSub(A.active, 1);
    A.st[h] = t;
    A.cnt[h] = 0;
}

// ranks, per-depth maxima and the capped count
__global__ void aca_stats_kernel(const AcaState *st, int64_t nint, int *rank, int *rmax,
                                 int *capped)
{
    int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (h >= nint)
        return;
    AcaState t = st[h];
    rank[h] = t.k;
    atomicMax(&rmax[depth_of_node(h) + 1], t.k);
    if (t.done == ACA_CAPPED)
        atomicAdd(capped, 1);
}

// zero columns [rank, rmax) of the panel on the rows of each chunk's block
__global__ void aca_pad_kernel(double *W, int64_t n, const Chunk *chunks, const int *rank,
                               const int *rmax, const int64_t *cofa)
{
    const Chunk ch = chunks[blockIdx.x];
    int d = depth_of_node(ch.node);
    int r0 = rank[ch.node], r1 = rmax[d + 1];
    int64_t col0 = cofa[d + 1];
    for (int c = r0; c < r1; ++c)
        for (int64_t g = ch.lo + threadIdx.x; g < ch.hi; g += blockDim.x)
            W[(col0 + c) * n + g] = 0.0;
}

void run_aca(Pipeline &P)
{
    const Plan &p = *P.plan;
    hipStream_t s = P.stream;
    P.rmax.assign(p.L + 2, 0);
    P.ranks.assign(p.nint, 0);
    P.capped = 0;
    if (p.L == 0)
        return;
    int *pinned = nullptr;
    HIP_TRY(hipHostMalloc((void **)&pinned, 64 * sizeof(int), hipHostMallocDefault));
    struct Guard {
        int *p;
        ~Guard() { (void)hipHostFree(p); }
    } g{pinned};
    int64_t *d_cofa = wsp<int64_t>(P, P.lay.misc);          // [0, 512): column offsets
    int *d_rmax = wsp<int>(P, P.lay.misc + 512);             // [512, 768): rmax per depth
    int *d_capped = wsp<int>(P, P.lay.misc + 768);
    HIP_TRY(hipMemcpyAsync(d_cofa, p.cofa.data(), sizeof(int64_t) * p.cofa.size(),
                           hipMemcpyHostToDevice, s));
    AcaArgs A;
    A.x = P.x;
    A.n = p.n;
    A.kp = P.kp;
    A.tol = P.tol;
    A.W = wsp<double>(P, P.lay.W);
    A.start = p.d_start;
    A.end = p.d_end;
    A.cofa = d_cofa;
    A.st = wsp<AcaState>(P, P.lay.aca_state);
    A.used = wsp<int>(P, P.lay.aca_used);
    A.vdots = wsp<double>(P, P.lay.aca_vdots);
    A.vstride = std::max(p.cap, 1);
    A.part = wsp<double>(P, P.lay.aca_part);
    A.pw = p.aca_pw;
    A.cnt = wsp<int>(P, P.lay.aca_cnt);
    A.active = wsp<int>(P, P.lay.aca_active);
    HIP_TRY(hipMemsetAsync(A.active, 0, 4 * sizeof(int), s));
    int nb = (int)((p.nint + 255) / 256);
    aca_init_kernel<<<nb, 256, 0, s>>>(A, p.nint, p.cap);
    HIP_TRY(hipGetLastError());
    AcaArgs R = A, C = A;
    R.chunks = p.d_aca_row;
    R.nch = p.d_aca_nrow;
    R.base = p.d_aca_rowbase;
    C.chunks = p.d_aca_col;
    C.nch = p.d_aca_ncol;
    C.base = p.d_aca_colbase;
    const int nrow = (int)p.aca_row.size(), ncol = (int)p.aca_col.size();
    const int max_iter = (p.cap + 1) * (ZERO_RETRY + 2) + 4;
    int it = 0;
    for (; it < max_iter; ++it) {
        if (nrow)
            aca_pass_kernel<true><<<nrow, ACA_THREADS, 0, s>>>(R);
        if (ncol)
            aca_pass_kernel<false><<<ncol, ACA_THREADS, 0, s>>>(C);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(pinned, A.active, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (pinned[0] <= 0)
            break;
    }
    if (it >= max_iter)
        throw Error{HODLR_EDEVICE, "cross approximation did not terminate"};
    int *rank = wsp<int>(P, P.lay.rank);
    HIP_TRY(hipMemsetAsync(d_rmax, 0, 68 * sizeof(int), s));
    aca_stats_kernel<<<nb, 256, 0, s>>>(A.st, p.nint, rank, d_rmax, d_capped);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(pinned, d_rmax, sizeof(int) * (p.L + 2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(pinned + 48, d_capped, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(P.ranks.data(), rank, sizeof(int) * p.nint, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int j = 0; j <= p.L + 1 && j < 48; ++j)
        P.rmax[j] = pinned[j];
    P.capped = pinned[48];
    // zero the padding columns of every block below its panel's maximum rank
    if (nrow)
        aca_pad_kernel<<<nrow, 256, 0, s>>>(A.W, p.n, p.d_aca_row, rank, d_rmax, d_cofa);
    if (ncol)
        aca_pad_kernel<<<ncol, 256, 0, s>>>(A.W, p.n, p.d_aca_col, rank, d_rmax, d_cofa);
    HIP_TRY(hipGetLastError());
}

}  // namespace hodlr
