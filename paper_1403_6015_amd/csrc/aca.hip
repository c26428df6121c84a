// Batched adaptive cross approximation (ACA) of every off-diagonal block
// K(alpha, beta) of the tree (§3.1 of the paper: an approximate partially
// pivoted LU that builds A ~ sum_k u_k v_k^T from rows and columns of A,
// with a sub-sampled error estimate).  Entries are evaluated on the fly from
// the ordered coordinates; u_k fills column k of the alpha rows and v_k
// column k of the beta rows of the depth-(d+1) panel.
//
// One step of the method (same rules as the oracle's walk-through):
//   v = A(i*, :) - sum_l u_l(i*) v_l;  j* = first argmax |v|;
//   v(j*) == 0: mark i* used, retry with the unused row nearest the split;
//   u = (A(:, j*) - sum_l v_l(j*) u_l) / v(j*);
//   ||S||_F^2 += |u|^2 |v|^2 + 2 sum_l (u.u_l)(v.v_l);
//   stop when |u| |v| <= tol ||S||_F or at the rank cap; otherwise the next
//   pivot row is the first argmax |u| over unused rows.
//
// Two paths, no communication between work-groups inside a launch (on this
// chip the L2 caches of the eight dies are not coherent, so intra-launch
// hand-offs would need device-wide cache write-backs):
//   * small blocks (both sides <= ACA_SMALL): one work-group runs the whole
//     loop for one block, all blocks in a single launch;
//   * large blocks: each step is a row pass and a column pass over all large
//     blocks, every work-group covering the plan's chunk of indices of one block.  Each
//     pass first re-derives the pivot and the norms from the previous pass's
//     per-work-group records (identically in every work-group of the block),
//     so state only moves across launch boundaries (double-buffered).
#include "common.h"

#include <cstring>

namespace hodlr {

// work-group size of the small-block path for blocks with a side above
// ACA_TINY; blocks with both sides <= ACA_TINY run on one wave (four entries
// per lane, wave reductions only).  Measured at n = 2^20: all blocks on 256
// threads 0.39 ms, on 128 threads 0.49 ms, on one wave 0.42 ms (32 entries
// per lane need 256 VGPRs); 256 threads plus one wave for the 128- and
// 256-point sides (6144 of the 7936 blocks) 0.22 ms; a third class (sides up
// to 512 on one wave, or up to 1024 on 128 threads) measured no faster.
constexpr int ACA_SMALL_TH = 256;


enum BigPhase { BP_FRESH = 0, BP_ROWDONE = 1, BP_COLDONE = 2, BP_RETRY = 3 };

struct AcaArgs {
    const double *x;
    int64_t n;
    KParams kp;
    double tol;
    double *W;
    const int64_t *start, *end;
    const int64_t *cofa;
    int cap;
};

__device__ __forceinline__ int depth_of_node(int64_t h)
{
    return 63 - __clzll((unsigned long long)(h + 1));
}

__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi)
{
    return v > bv || (v == bv && i < bi);
}

// block argmax over NW waves (ties to the smaller index) carrying the signed
// value; every thread returns the result
template <int NW>
__device__ void block_argmax(double &v, int64_t &i, double &sgn, double *rv, int64_t *ri,
                             double *rs)
{
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    wave_argmax_signed(v, i, sgn);
    if (lane == 0) {
        rv[wid] = v;
        ri[wid] = i;
        rs[wid] = sgn;
    }
    __syncthreads();
    v = rv[0];
    i = ri[0];
    sgn = rs[0];
    for (int w = 1; w < NW; ++w)
        if (better(rv[w], ri[w], v, i)) {
            v = rv[w];
            i = ri[w];
            sgn = rs[w];
        }
    __syncthreads();
}

template <int NW>
__device__ double block_sum(double v, double *red)
{
    static_assert(NW == 2 || NW == 4, "two or four waves");
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    v = wave_sum(v);
    if (lane == 0)
        red[wid] = v;
    __syncthreads();
    double s = (NW == 4) ? (red[0] + red[1]) + (red[2] + red[3]) : red[0] + red[1];
    __syncthreads();
    return s;
}

// reductions over a work-group of TH threads: one wave needs no LDS or barrier
template <int TH>
__device__ __forceinline__ void grp_argmax(double &v, int64_t &i, double &sgn, double *rv,
                                           int64_t *ri, double *rs)
{
    if constexpr (TH == 64)
        wave_argmax_signed(v, i, sgn);
    else
        block_argmax<TH / 64>(v, i, sgn, rv, ri, rs);
}

template <int TH>
__device__ __forceinline__ double grp_sum(double v, double *red)
{
    if constexpr (TH == 64)
        return wave_sum(v);
    else
        return block_sum<TH / 64>(v, red);
}

// ------------------------------------------------------------ small blocks
struct SmallArgs {
    AcaArgs a;
    const int *nodes;   // internal nodes handled here
    int *rank;
    int *status;        // per node AcaDone
};

// RB bounds the rank (LDS arrays); a plan with max_rank <= RMAX_LDS uses the
// narrow variant, whose LDS footprint keeps more work-groups per CU
template <int TH, int MAXS, int RB>
__global__ __launch_bounds__(TH) void aca_small_kernel(SmallArgs S)
{
    const AcaArgs &A = S.a;
    const int64_t h = S.nodes[blockIdx.x];
    constexpr int EPT = MAXS / TH;   // entries per thread (block sides <= MAXS)
    const int tid = threadIdx.x;
    const int64_t s = A.start[h], e = A.end[h], m = s + (e - s) / 2;
    const int64_t na = m - s, nb = e - m, n = A.n;
    const int64_t col0 = A.cofa[depth_of_node(h) + 1];
    double *__restrict__ W = A.W;
    __shared__ double rv[4], rs[4], red[4];
    __shared__ int64_t ri[4];
    __shared__ double sfix[RB];
    __shared__ double vdot[RB];
    __shared__ unsigned char used[MAXS];
    const int64_t full = na < nb ? na : nb;
    const int cap = (int)(A.cap < full ? A.cap : full);
    const bool usercap = A.cap < full;
    for (int64_t i = tid; i < na; i += TH)
        used[i] = 0;
    __syncthreads();
    int k = 0, zeros = 0, nused = 0, done = (cap <= 0) ? ACA_EXHAUSTED : ACA_ACTIVE;
    int64_t istar = na - 1;
    double s2 = 0.0;
    double uv[EPT];
    while (done == ACA_ACTIVE) {
        // residual row at i*
        // (written by other threads of this work-group: read past the L1)
        for (int l = tid; l < k; l += TH)
            sfix[l] = ld_coherent(&W[(col0 + l) * n + s + istar]);
        __syncthreads();
        double bv = -1.0, bs = 0.0, sq = 0.0;
        int64_t bi = INT64_MAX;
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            int64_t j = tid + (int64_t)t * TH;
            uv[t] = 0.0;
            if (j < nb) {
                double a = kentry(A.kp, A.x, n, s + istar, m + j);
                for (int l = 0; l < k; ++l)
                    a -= sfix[l] * W[(col0 + l) * n + m + j];
                W[(col0 + k) * n + m + j] = a;
                uv[t] = a;
                sq += a * a;
                if (fabs(a) > bv) {
                    bv = fabs(a);
                    bs = a;
                    bi = j;
                }
            }
        }
        grp_argmax<TH>(bv, bi, bs, rv, ri, rs);
        if (tid == 0)
            used[istar] = 1;
        ++nused;
        __syncthreads();
        if (bv == 0.0) {
            ++zeros;
            if (zeros > ZERO_RETRY || nused >= na) {
                done = ACA_EXHAUSTED;
            } else {
                int64_t c = na - 1;
                while (c >= 0 && used[c])
                    --c;
                istar = c;
            }
            continue;
        }
        zeros = 0;
        const double v2 = grp_sum<TH>(sq, red);
        for (int l = 0; l < k; ++l) {
            double d = 0.0;
#pragma unroll
            for (int t = 0; t < EPT; ++t) {
                int64_t j = tid + (int64_t)t * TH;
                if (j < nb)
                    d += uv[t] * W[(col0 + l) * n + m + j];
            }
            d = grp_sum<TH>(d, red);
            if (tid == 0)
                vdot[l] = d;
        }
        // residual column at j*
        const int64_t jstar = bi;
        const double delta = bs;
        for (int l = tid; l < k; l += TH)
            sfix[l] = ld_coherent(&W[(col0 + l) * n + m + jstar]);
        __syncthreads();
        bv = -1.0;
        bs = 0.0;
        bi = INT64_MAX;
        sq = 0.0;
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            int64_t i = tid + (int64_t)t * TH;
            uv[t] = 0.0;
            if (i < na) {
                double a = kentry(A.kp, A.x, n, s + i, m + jstar);
                for (int l = 0; l < k; ++l)
                    a -= sfix[l] * W[(col0 + l) * n + s + i];
                a = a / delta;
                W[(col0 + k) * n + s + i] = a;
                uv[t] = a;
                sq += a * a;
                if (!used[i] && fabs(a) > bv) {
                    bv = fabs(a);
                    bs = a;
                    bi = i;
                }
            }
        }
        grp_argmax<TH>(bv, bi, bs, rv, ri, rs);
        const double u2 = grp_sum<TH>(sq, red);
        double cross = 0.0;
        for (int l = 0; l < k; ++l) {
            double d = 0.0;
#pragma unroll
            for (int t = 0; t < EPT; ++t) {
                int64_t i = tid + (int64_t)t * TH;
                if (i < na)
                    d += uv[t] * W[(col0 + l) * n + s + i];
            }
            d = grp_sum<TH>(d, red);
            cross += d * vdot[l];
        }
        s2 += u2 * v2 + 2.0 * cross;
        k += 1;
        if (sqrt(u2) * sqrt(v2) <= A.tol * sqrt(s2 > 0.0 ? s2 : 0.0))
            done = ACA_CONVERGED;
        else if (k >= cap)
            done = usercap ? ACA_CAPPED : ACA_CONVERGED;
        else if (nused >= na || bv < 0.0)
            done = ACA_EXHAUSTED;
        else
            istar = bi;
    }
    if (tid == 0) {
        S.rank[h] = k;
        S.status[h] = done;
    }
}

// ------------------------------------------------------------ batched form
// Whole cross approximation of one block (any size) in one work-group, for
// every internal node of every batch item (item = blockIdx.z).  Used rows are
// kept as a list in LDS; the dots with earlier terms re-read the panel
// entries the same thread wrote.
template <int RB>
__global__ __launch_bounds__(ACA_THREADS) void aca_block_kernel(AcaArgs A0, BatchArgs B, int *rank0,
                                                               int *status0)
{
    const int it = blockIdx.z;
    const int64_t h = blockIdx.x;
    const int tid = threadIdx.x;
    const KParams kp = item_kp(A0.kp, B, it);
    double *__restrict__ W = ioff(A0.W, B, it);
    int *rank = ioff(rank0, B, it);
    int *status = ioff(status0, B, it);
    const int64_t s = A0.start[h], e = A0.end[h], m = s + (e - s) / 2;
    const int64_t na = m - s, nb = e - m, n = A0.n;
    const int64_t col0 = A0.cofa[depth_of_node(h) + 1];
    __shared__ double rv[4], rs[4], red[4];
    __shared__ int64_t ri[4];
    constexpr int UM = used_max(RB);
    __shared__ double sfix[RB];
    __shared__ double vdot[RB];
    __shared__ int usedl[UM];
    const int64_t full = na < nb ? na : nb;
    const int cap = (int)(A0.cap < full ? A0.cap : full);
    const bool usercap = A0.cap < full;
    int k = 0, zeros = 0, nused = 0, done = (cap <= 0) ? ACA_EXHAUSTED : ACA_ACTIVE;
    int64_t istar = na - 1;
    double s2 = 0.0;
    while (done == ACA_ACTIVE) {
        for (int l = tid; l < k; l += ACA_THREADS)
            sfix[l] = ld_coherent(&W[(col0 + l) * n + s + istar]);
        __syncthreads();
        double bv = -1.0, bs = 0.0, sq = 0.0;
        int64_t bi = INT64_MAX;
        for (int64_t j = tid; j < nb; j += ACA_THREADS) {
            double a = kentry(kp, A0.x, n, s + istar, m + j);
            for (int l = 0; l < k; ++l)
                a -= sfix[l] * W[(col0 + l) * n + m + j];
            W[(col0 + k) * n + m + j] = a;
            sq += a * a;
            if (fabs(a) > bv) {
                bv = fabs(a);
                bs = a;
                bi = j;
            }
        }
        block_argmax<ACA_THREADS / 64>(bv, bi, bs, rv, ri, rs);
        if (tid == 0 && nused < UM)
            usedl[nused] = (int)istar;
        ++nused;
        __syncthreads();
        if (bv == 0.0) {
            ++zeros;
            if (zeros > ZERO_RETRY || nused >= na || nused >= UM) {
                done = ACA_EXHAUSTED;
            } else {
                int64_t c = na - 1;
                for (; c >= 0; --c) {
                    bool u = false;
                    for (int q = 0; q < nused; ++q)
                        u = u || (usedl[q] == c);
                    if (!u)
                        break;
                }
                istar = c;
            }
            continue;
        }
        zeros = 0;
        const double v2 = block_sum<ACA_THREADS / 64>(sq, red);
        for (int l = 0; l < k; ++l) {
            double d = 0.0;
            for (int64_t j = tid; j < nb; j += ACA_THREADS)
                d += W[(col0 + k) * n + m + j] * W[(col0 + l) * n + m + j];
            d = block_sum<ACA_THREADS / 64>(d, red);
            if (tid == 0)
                vdot[l] = d;
        }
        const int64_t jstar = bi;
        const double delta = bs;
        for (int l = tid; l < k; l += ACA_THREADS)
            sfix[l] = ld_coherent(&W[(col0 + l) * n + m + jstar]);
        __syncthreads();
        bv = -1.0;
        bs = 0.0;
        bi = INT64_MAX;
        sq = 0.0;
        for (int64_t i = tid; i < na; i += ACA_THREADS) {
            double a = kentry(kp, A0.x, n, s + i, m + jstar);
            for (int l = 0; l < k; ++l)
                a -= sfix[l] * W[(col0 + l) * n + s + i];
            a = a / delta;
            W[(col0 + k) * n + s + i] = a;
            sq += a * a;
            bool elig = true;
            for (int q = 0; q < nused && q < UM; ++q)
                elig = elig && (usedl[q] != (int)i);
            if (elig && fabs(a) > bv) {
                bv = fabs(a);
                bs = a;
                bi = i;
            }
        }
        block_argmax<ACA_THREADS / 64>(bv, bi, bs, rv, ri, rs);
        const double u2 = block_sum<ACA_THREADS / 64>(sq, red);
        double cross = 0.0;
        for (int l = 0; l < k; ++l) {
            double d = 0.0;
            for (int64_t i = tid; i < na; i += ACA_THREADS)
                d += W[(col0 + k) * n + s + i] * W[(col0 + l) * n + s + i];
            d = block_sum<ACA_THREADS / 64>(d, red);
            cross += d * vdot[l];
        }
        s2 += u2 * v2 + 2.0 * cross;
        k += 1;
        if (sqrt(u2) * sqrt(v2) <= A0.tol * sqrt(s2 > 0.0 ? s2 : 0.0))
            done = ACA_CONVERGED;
        else if (k >= cap)
            done = usercap ? ACA_CAPPED : ACA_CONVERGED;
        else if (nused >= na || nused >= UM || bv < 0.0)
            done = ACA_EXHAUSTED;
        else
            istar = bi;
    }
    if (tid == 0) {
        rank[h] = k;
        status[h] = done;
    }
}

// per item: rank maxima per depth (into the item's own area and, by atomic
// maximum, into the batch-wide area of item 0) and the capped count
__global__ __launch_bounds__(256) void aca_batch_stats_kernel(const int *rank0, const int *status0,
                                                              int64_t nint, BatchArgs B, int *rmax0,
                                                              int *capped0, int *rmax_all,
                                                              int *capped_all)
{
    const int it = blockIdx.z;
    const int *rank = ioff(rank0, B, it);
    const int *status = ioff(status0, B, it);
    int *rmax = ioff(rmax0, B, it);
    int *capped = ioff(capped0, B, it);
    __shared__ int smax[64];
    __shared__ int scap;
    if (threadIdx.x < 64)
        smax[threadIdx.x] = 0;
    if (threadIdx.x == 0)
        scap = 0;
    __syncthreads();
    int mycap = 0;
    for (int64_t h = threadIdx.x; h < nint; h += 256) {
        atomicMax(&smax[depth_of_node(h) + 1], rank[h]);
        mycap += (status[h] == ACA_CAPPED) ? 1 : 0;
    }
    atomicAdd(&scap, mycap);
    __syncthreads();
    if (threadIdx.x < 64) {
        rmax[threadIdx.x] = smax[threadIdx.x];
        atomicMax(&rmax_all[threadIdx.x], smax[threadIdx.x]);
    }
    if (threadIdx.x == 0) {
        *capped = scap;
        atomicAdd(capped_all, scap);
    }
}

// zero panel columns [rank, rmax_all) of every block of every item
__global__ void aca_batch_pad_kernel(double *W0, int64_t n, const Chunk *chunks, const int *rank0,
                                     const int *rmax_all, const int64_t *cofa, BatchArgs B)
{
    const int it = blockIdx.z;
    double *W = ioff(W0, B, it);
    const int *rank = ioff(rank0, B, it);
    const Chunk ch = chunks[blockIdx.x];
    int d = depth_of_node(ch.node);
    int r0 = rank[ch.node], r1 = rmax_all[d + 1];
    int64_t col0 = cofa[d + 1];
    for (int c = r0; c < r1; ++c)
        for (int64_t g = ch.lo + threadIdx.x; g < ch.hi; g += blockDim.x)
            W[(col0 + c) * n + g] = 0.0;
}

// Batched compression: one launch for every block of every item, then the
// batch-wide rank maxima (the common column layout) come back to the host.
void run_aca_batched(Pipeline &P)
{
    const Plan &p = *P.plan;
    hipStream_t s = P.stream;
    P.rmax.assign(p.L + 2, 0);
    P.ranks.clear();
    P.capped = 0;
    if (p.L == 0)
        return;
    int64_t *d_cofa = wsp<int64_t>(P, P.lay.misc);   // item 0 holds the shared copy
    int *d_rmax = wsp<int>(P, P.lay.misc + 512);
    int *d_capped = wsp<int>(P, P.lay.misc + 784);
    int *d_rmax_all = wsp<int>(P, P.lay.misc + 1536);
    int *d_capped_all = wsp<int>(P, P.lay.misc + 1536 + 256);
    HIP_TRY(hipMemcpyAsync(d_cofa, p.cofa.data(), sizeof(int64_t) * p.cofa.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(d_rmax_all, 0, 320, s));
    AcaArgs A;
    A.x = P.x;
    A.n = p.n;
    A.kp = P.kp;
    A.tol = P.tol;
    A.W = wsp<double>(P, P.lay.W);
    A.start = p.d_start;
    A.end = p.d_end;
    A.cofa = d_cofa;
    A.cap = p.cap;
    int *rank = wsp<int>(P, P.lay.rank);
    int *status = wsp<int>(P, P.lay.aca_status);
    {
        ProfScope ps(s, PS_ACA_SMALL);
        const dim3 grid((unsigned)p.nint, 1, P.nitems);
        if (p.cap <= RMAX_LDS)
            aca_block_kernel<RMAX_LDS><<<grid, ACA_THREADS, 0, s>>>(A, P.batch, rank, status);
        else
            aca_block_kernel<RMAX_ABS><<<grid, ACA_THREADS, 0, s>>>(A, P.batch, rank, status);
    }
    {
        ProfScope ps(s, PS_ACA_MISC);
        aca_batch_stats_kernel<<<dim3(1, 1, P.nitems), 256, 0, s>>>(
            rank, status, p.nint, P.batch, d_rmax, d_capped, d_rmax_all, d_capped_all);
    }
    HIP_TRY(hipGetLastError());
    int host[80];
    HIP_TRY(hipMemcpyAsync(host, d_rmax_all, sizeof(int) * 65, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int j = 0; j <= p.L + 1 && j < 64; ++j)
        P.rmax[j] = host[j];
    P.capped = host[64];
    ProfScope ps(s, PS_ACA_MISC);
    if (!p.pad_chunks.empty())
        aca_batch_pad_kernel<<<dim3((unsigned)p.pad_chunks.size(), 1, P.nitems), 256, 0, s>>>(
            A.W, p.n, p.d_pad_chunks, rank, d_rmax_all, d_cofa, P.batch);
    HIP_TRY(hipGetLastError());
}

// ------------------------------------------------------------ large blocks
struct BigArgs {
    AcaArgs a;
    const Chunk *chunks;      // this pass's chunks (rows of beta or of alpha)
    const int *bnode;         // per big-block index: heap index
    const int *pnch, *pbase;  // previous pass's records: count and first slot per big block
    const int *cidx;          // per chunk: big-block index
    const BigState *sin;
    BigState *sout;
    const double *pin;        // previous pass's records
    double *pout;             // this pass's records
    int pw;
    int *used;                // per big block, USED_MAX rows
    double *vdots;            // per big block, RMAX_ABS
    int *ndone;
};

__global__ void aca_big_init_kernel(BigState *st, const int *bnode, int nbig, AcaArgs A)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbig)
        return;
    int64_t h = bnode[b];
    int64_t s = A.start[h], e = A.end[h], m = s + (e - s) / 2;
    int64_t na = m - s, nb = e - m, full = na < nb ? na : nb;
    BigState t;
    t.k = 0;
    t.istar = (int)(na - 1);
    t.jstar = 0;
    t.zeros = 0;
    t.nused = 0;
    t.cap = (int)(A.cap < full ? A.cap : full);
    t.usercap = A.cap < full;
    t.done = t.cap <= 0 ? ACA_EXHAUSTED : ACA_ACTIVE;
    t.phase = BP_FRESH;
    t.pad_ = 0;
    t.delta = t.v2 = t.s2 = 0.0;
    st[b] = t;
}

// Reduce the previous pass's records of one big block: slot 0 = max |value|
// (over eligible indices), 1 = its index, 2 = squared norm, 3 = signed value,
// 4 + l = dot with term l.  Every thread ends with the same results.
// Combine the previous pass's per-work-group records of one block: the sums
// of slots 4 + l (l < k) and of slot 2 into dots[0..k], and the argmax of
// slot 0 (index in slot 1, signed value in slot 3).  One sweep over the
// records: the first RR_REG sums and the argmax stay in registers and are
// reduced together behind one barrier; sums beyond RR_REG (ranks above it)
// follow RR_REG at a time, each group behind one barrier pair.
constexpr int RR_REG = 8;

__device__ void reduce_records(const double *rec, int nrec, int pw, int k, double *dots,
                               double &bv, int64_t &bi, double &bs, double *rv, int64_t *ri,
                               double *rs, double (*sred)[RR_REG + 1])
{
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kr = k < RR_REG ? k : RR_REG;
    double acc[RR_REG + 1];
#pragma unroll
    for (int l = 0; l <= RR_REG; ++l)
        acc[l] = 0.0;
    bv = -1.0;
    bs = 0.0;
    bi = INT64_MAX;
    for (int c = tid; c < nrec; c += ACA_THREADS) {
        // a record's words all issued together: slots past the k terms are
        // read at slot 4 (always present) and dropped, so no load waits
        // behind a branch
        const double *r = rec + (int64_t)c * pw;
        double rr[RR_REG];
#pragma unroll
        for (int l = 0; l < RR_REG; ++l)
            rr[l] = r[4 + (l < kr ? l : 0)];
        const double v = r[0], di = r[1], sv = r[3];
        acc[RR_REG] += r[2];
#pragma unroll
        for (int l = 0; l < RR_REG; ++l)
            acc[l] += l < kr ? rr[l] : 0.0;
        const int64_t i = di < 0.0 ? INT64_MAX : (int64_t)di;
        if (better(v, i, bv, bi)) {
            bv = v;
            bi = i;
            bs = sv;
        }
    }
#pragma unroll
    for (int l = 0; l <= RR_REG; ++l)
        if (l < kr || l == RR_REG) {
            const double w = wave_sum(acc[l]);
            if (lane == 0)
                sred[wid][l] = w;
        }
    // the argmax ends with a barrier, after which sred is complete
    block_argmax<ACA_THREADS / 64>(bv, bi, bs, rv, ri, rs);
    if (tid <= kr) {
        const int l = (tid == kr) ? RR_REG : tid;
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < ACA_THREADS / 64; ++w)
            t += sred[w][l];
        dots[tid == kr ? k : tid] = t;
    }
    // the remaining terms RR_REG at a time: their loads in flight together
    // and one barrier pair per group instead of per term (same summation
    // order as a block_sum per term)
    if (k > RR_REG)
        __syncthreads();   // sred read above before it is refilled
    for (int l0 = RR_REG; l0 < k; l0 += RR_REG) {
        const int kl = k - l0 < RR_REG ? k - l0 : RR_REG;
        double a[RR_REG];
#pragma unroll
        for (int j = 0; j < RR_REG; ++j)
            a[j] = 0.0;
        for (int c = tid; c < nrec; c += ACA_THREADS) {
            const double *r = rec + (int64_t)c * pw + 4 + l0;
            double rr[RR_REG];
#pragma unroll
            for (int j = 0; j < RR_REG; ++j)
                rr[j] = r[j < kl ? j : 0];
#pragma unroll
            for (int j = 0; j < RR_REG; ++j)
                a[j] += j < kl ? rr[j] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < RR_REG; ++j)
            if (j < kl) {
                const double w = wave_sum(a[j]);
                if (lane == 0)
                    sred[wid][j] = w;
            }
        __syncthreads();
        if (tid < kl) {
            static_assert(ACA_THREADS == 256, "four waves");
            dots[l0 + tid] = (sred[0][tid] + sred[1][tid]) + (sred[2][tid] + sred[3][tid]);
        }
        __syncthreads();   // sred free for the next group
    }
    __syncthreads();   // dots[] visible
}

// Terms read per round in residual_terms and term_dots: RT * EPT loads in
// flight per thread. With few entries per thread one term at a time leaves a
// pass with k = 64 waiting on 64 dependent round trips per entry; with 8
// entries per thread eight terms per round raise the kernel from 54 to 171
// VGPRs and its occupancy from 8 to 2 waves per SIMD.
template <int EPT>
constexpr int terms_per_round() { return EPT >= 8 ? 1 : 16 / EPT; }

// val[q] -= sum over the k earlier terms of sfix[l] W[l][g_q] (g_q the
// thread's entries of the chunk), in order of l
template <int EPT>
__device__ __forceinline__ void residual_terms(const double *__restrict__ W, int64_t n, int64_t col0,
                                               int k, const double *sfix, const Chunk &ch, int tid,
                                               double (&val)[EPT])
{
    constexpr int RT = terms_per_round<EPT>();
    for (int l0 = 0; l0 < k; l0 += RT) {
        // every load of the round issued unconditionally (term index and row
        // clamped into the block's written entries), the dropped ones zeroed
        // after: a conditional load would wait in its own branch
        double w[RT][EPT];
#pragma unroll
        for (int u = 0; u < RT; ++u)
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
                const int64_t gc = g < ch.hi ? g : ch.hi - 1;
                const int lu = l0 + u < k ? l0 + u : k - 1;
                w[u][q] = W[(col0 + lu) * n + gc];
            }
#pragma unroll
        for (int u = 0; u < RT; ++u)
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
                asm volatile("" : "+v"(w[u][q]));
                w[u][q] = (l0 + u < k && g < ch.hi) ? w[u][q] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < RT; ++u)
            if (l0 + u < k)
#pragma unroll
                for (int q = 0; q < EPT; ++q)
                    val[q] -= sfix[l0 + u] * w[u][q];
    }
}

// sdot[wave][l] = this wave's part of sum_g val_g W[l][g] for l < k, RT terms
// at a time (their loads and wave sums independent of each other)
template <int EPT, int RB>
__device__ __forceinline__ void term_dots(const double *__restrict__ W, int64_t n, int64_t col0, int k,
                                          const Chunk &ch, int tid, const double (&val)[EPT],
                                          double (*sdot)[RB + 1])
{
    constexpr int RT = terms_per_round<EPT>();
    const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int l0 = 0; l0 < k; l0 += RT) {
        double d[RT];
#pragma unroll
        for (int u = 0; u < RT; ++u) {
            d[u] = 0.0;
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                // clamped and unconditional; val is 0 past the chunk, and a
                // term past k is never stored
                const int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
                const int64_t gc = g < ch.hi ? g : ch.hi - 1;
                const int lu = l0 + u < k ? l0 + u : k - 1;
                d[u] += val[q] * W[(col0 + lu) * n + gc];
            }
        }
#pragma unroll
        for (int u = 0; u < RT; ++u)
            d[u] = wave_sum(d[u]);
        if (lane == 0)
#pragma unroll
            for (int u = 0; u < RT; ++u)
                if (l0 + u < k)
                    sdot[wid][l0 + u] = d[u];
    }
}

// Kernel entries K(fix, g) for the thread's EPT rows g = lo + tid + 256 q of
// the chunk (0 past it), the same values as kentry: every coordinate load is
// issued (rows clamped into the chunk) before the first entry is formed, so
// the rows do not take one memory round trip each.
template <int EPT>
__device__ __forceinline__ void chunk_entries(const KParams &kp, const double *__restrict__ x,
                                              int64_t n, int64_t fix, const Chunk &ch, int tid,
                                              double (&val)[EPT])
{
    if (kp.dim == 1) {
        const double xf = x[fix];
        double xg[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
            xg[q] = x[g < ch.hi ? g : ch.hi - 1];
        }
#pragma unroll
        for (int q = 0; q < EPT; ++q)
            asm volatile("" : "+v"(xg[q]));
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
            const double t = xg[q] - xf;
            const double v = kfun_r2<double>(kp.kind, kp.a2, kp.c, 0.0 + t * t);
            val[q] = g < ch.hi ? v : 0.0;
        }
        return;
    }
    if constexpr (EPT > 2) {
        // plans give 2048-entry chunks (EPT 8) to 1-D points only; any other
        // case takes the entries one by one, keeping these registers free
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
            const double v = kentry(kp, x, n, fix, g < ch.hi ? g : ch.hi - 1);
            val[q] = g < ch.hi ? v : 0.0;
        }
        return;
    }
    double xf[3], xg[EPT][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        xf[d] = x[(d < kp.dim ? d : 0) * n + fix];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
        const int64_t gc = g < ch.hi ? g : ch.hi - 1;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            xg[q][d] = x[(d < kp.dim ? d : 0) * n + gc];
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q)
#pragma unroll
        for (int d = 0; d < 3; ++d)
            asm volatile("" : "+v"(xg[q][d]));
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
        double r2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double t = xg[q][d] - xf[d];
            r2 += d < kp.dim ? t * t : 0.0;
        }
        const double v = kfun_r2<double>(kp.kind, kp.a2, kp.c, r2);
        val[q] = g < ch.hi ? v : 0.0;
    }
}

template <bool ROW, int EPT, int RB>
__global__ __launch_bounds__(ACA_THREADS) void aca_big_pass_kernel(BigArgs B)
{
    const AcaArgs &A = B.a;
    const Chunk ch = B.chunks[blockIdx.x];
    const int b = B.cidx[blockIdx.x];
    const int64_t h = B.bnode[b];
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    __shared__ double rv[4], rs[4];
    __shared__ int64_t ri[4];
    // the block's used-row list lives in HBM with room for RMAX_ABS terms; a
    // block capped at RB needs at most used_max(RB) of its entries
    constexpr int UM = used_max(RB);
    __shared__ double sfix[RB];
    __shared__ double dots[RB + 1];
    __shared__ double sdot[4][RB + 1];
    __shared__ double sred[ACA_THREADS / 64][RR_REG + 1];
    __shared__ int sused[UM];
    BigState t = B.sin[b];
    const int64_t s = A.start[h], e = A.end[h], m = s + (e - s) / 2;
    const int64_t na = m - s, n = A.n;
    const bool lead = ch.lo == (ROW ? m : s);   // the block's first chunk writes its state
    const int64_t col0 = A.cofa[depth_of_node(h) + 1];
    double *__restrict__ W = A.W;
    int *used = B.used + (int64_t)b * USED_MAX;
    const double *prec = B.pin + (int64_t)B.pbase[b] * B.pw;
    const int pn = B.pnch[b];
    if (t.done != ACA_ACTIVE) {
        if (lead && tid == 0)
            B.sout[b] = t;
        return;
    }
    if (ROW) {
        if (t.phase == BP_COLDONE) {
            // finish the previous step from the column records
            double bv, bs;
            int64_t bi;
            reduce_records(prec, pn, B.pw, t.k, dots, bv, bi, bs, rv, ri, rs, sred);
            double u2 = dots[t.k];
            double cross = 0.0;
            for (int l = 0; l < t.k; ++l)
                cross += dots[l] * B.vdots[(int64_t)b * RMAX_ABS + l];
            t.s2 += u2 * t.v2 + 2.0 * cross;
            t.k += 1;
            double s2 = t.s2 > 0.0 ? t.s2 : 0.0;
            if (sqrt(u2) * sqrt(t.v2) <= A.tol * sqrt(s2))
                t.done = ACA_CONVERGED;
            else if (t.k >= t.cap)
                t.done = t.usercap ? ACA_CAPPED : ACA_CONVERGED;
            else if (t.nused >= na || t.nused >= UM || bv < 0.0)
                t.done = ACA_EXHAUSTED;
            else
                t.istar = (int)(bi - s);
            if (t.done != ACA_ACTIVE) {
                if (lead && tid == 0) {
                    B.sout[b] = t;
                    atomicAdd(B.ndone, 1);
                }
                return;
            }
        }
        // evaluate the residual row i*; the row becomes used
        const int k = t.k;
        const int64_t fix = s + t.istar;
        for (int l = tid; l < k; l += ACA_THREADS)
            sfix[l] = W[(col0 + l) * n + fix];
        __syncthreads();
        double val[EPT];
        double bv = -1.0, bs = 0.0, sq = 0.0;
        int64_t bi = INT64_MAX;
        chunk_entries<EPT>(A.kp, A.x, n, fix, ch, tid, val);
        residual_terms<EPT>(W, n, col0, k, sfix, ch, tid, val);
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
            if (g < ch.hi) {
                const double a = val[q];
                W[(col0 + k) * n + g] = a;
                sq += a * a;
                if (fabs(a) > bv) {
                    bv = fabs(a);
                    bs = a;
                    bi = g;
                }
            }
        }
        term_dots<EPT, RB>(W, n, col0, k, ch, tid, val, sdot);
        sq = wave_sum(sq);
        if (lane == 0)
            sdot[wid][k] = sq;
        block_argmax<ACA_THREADS / 64>(bv, bi, bs, rv, ri, rs);
        double *rec = B.pout + (int64_t)ch.part * B.pw;
        if (tid == 0) {
            rec[0] = bv;
            rec[1] = (bi == INT64_MAX) ? -1.0 : (double)bi;
            rec[2] = (sdot[0][k] + sdot[1][k]) + (sdot[2][k] + sdot[3][k]);
            rec[3] = bs;
        }
        for (int l = tid; l < k; l += ACA_THREADS)
            rec[4 + l] = (sdot[0][l] + sdot[1][l]) + (sdot[2][l] + sdot[3][l]);
        if (lead && tid == 0) {
            if (t.nused < UM)
                used[t.nused] = t.istar;
            t.nused += 1;
            t.phase = BP_ROWDONE;
            B.sout[b] = t;
        }
        return;
    }
    // ---- column pass: pick the pivot column from the row records
    double bv, bs;
    int64_t bi;
    reduce_records(prec, pn, B.pw, t.k, dots, bv, bi, bs, rv, ri, rs, sred);
    const int nu = t.nused < UM ? t.nused : UM;
    for (int q = tid; q < nu; q += ACA_THREADS)
        sused[q] = used[q];
    __syncthreads();
    if (bv == 0.0) {
        if (lead && tid == 0) {
            t.zeros += 1;
            if (t.zeros > ZERO_RETRY || t.nused >= na || t.nused >= UM) {
                t.done = ACA_EXHAUSTED;
                atomicAdd(B.ndone, 1);
            } else {
                int c = (int)na - 1;
                for (; c >= 0; --c) {
                    bool u = false;
                    for (int q = 0; q < nu; ++q)
                        u = u || (sused[q] == c);
                    if (!u)
                        break;
                }
                t.istar = c;
                t.phase = BP_RETRY;
            }
            B.sout[b] = t;
        }
        return;
    }
    const int k = t.k;
    t.zeros = 0;
    t.jstar = (int)(bi - m);
    t.delta = bs;
    t.v2 = dots[k];
    const int64_t fix = bi;
    for (int l = tid; l < k; l += ACA_THREADS)
        sfix[l] = W[(col0 + l) * n + fix];
    __syncthreads();
    double val[EPT];
    double cv = -1.0, cs = 0.0, sq = 0.0;
    int64_t ci = INT64_MAX;
    chunk_entries<EPT>(A.kp, A.x, n, fix, ch, tid, val);
    residual_terms<EPT>(W, n, col0, k, sfix, ch, tid, val);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        int64_t g = ch.lo + tid + (int64_t)q * ACA_THREADS;
        if (g < ch.hi) {
            const double a = val[q] / t.delta;
            W[(col0 + k) * n + g] = a;
            val[q] = a;
            sq += a * a;
            int li = (int)(g - s);
            bool elig = true;
            for (int p = 0; p < nu; ++p)
                elig = elig && (sused[p] != li);
            if (elig && fabs(a) > cv) {
                cv = fabs(a);
                cs = a;
                ci = g;
            }
        }
    }
    term_dots<EPT, RB>(W, n, col0, k, ch, tid, val, sdot);
    sq = wave_sum(sq);
    if (lane == 0)
        sdot[wid][k] = sq;
    block_argmax<ACA_THREADS / 64>(cv, ci, cs, rv, ri, rs);
    double *rec = B.pout + (int64_t)ch.part * B.pw;
    if (tid == 0) {
        rec[0] = cv;
        rec[1] = (ci == INT64_MAX) ? -1.0 : (double)ci;
        rec[2] = (sdot[0][k] + sdot[1][k]) + (sdot[2][k] + sdot[3][k]);
        rec[3] = cs;
    }
    for (int l = tid; l < k; l += ACA_THREADS)
        rec[4 + l] = (sdot[0][l] + sdot[1][l]) + (sdot[2][l] + sdot[3][l]);
    if (lead && tid == 0) {
        for (int l = 0; l < k; ++l)
            B.vdots[(int64_t)b * RMAX_ABS + l] = dots[l];
        t.phase = BP_COLDONE;
        B.sout[b] = t;
    }
}

__global__ void aca_big_finish_kernel(const BigState *st, const int *bnode, int nbig, int *rank,
                                      int *status)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbig)
        return;
    rank[bnode[b]] = st[b].k;
    status[bnode[b]] = st[b].done;
}

// ranks, per-depth maxima and the capped count: one work-group.  Depth d's
// nodes are the heap range [2^d - 1, 2^(d+1) - 1); each thread keeps one
// maximum per depth in a register (the depth loop is unrolled, so no load
// waits on another depth's), then one wave reduction and one LDS atomic per
// wave and depth.  rmax[48] receives the capped count and rmax[49] the
// finished large-block count (ndone, when given), so that one copy of 64
// ints carries every statistic.
constexpr int STATS_DEPTHS = 46;   // depths 0 .. 45 (plans have at most 62 levels; ranks
                                   // beyond depth 45 would need more than 2^46 points)

__global__ __launch_bounds__(256) void aca_stats_kernel(const int *rank, const int *status,
                                                        int64_t nint, int *rmax, const int *ndone)
{
    // one flat pass: thread t reads blocks t + 256 u in rounds of 16, all of
    // a round's loads issued together (indices clamped, the tail masked
    // afterwards); its running maximum goes to the depth's LDS slot whenever
    // the depth changes (blocks in heap order, depth nondecreasing)
    constexpr int U = 16;
    __shared__ int smax[64];
    __shared__ int scap;
    if (threadIdx.x < 64)
        smax[threadIdx.x] = 0;
    if (threadIdx.x == 0)
        scap = 0;
    __syncthreads();
    int mycap = 0, cd = -1, cm = 0;
    for (int64_t h0 = threadIdx.x; h0 < nint; h0 += 256 * U) {
        int rv[U], sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t h = std::min<int64_t>(h0 + 256 * u, nint - 1);
            rv[u] = rank[h];
            sv[u] = status[h];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            asm volatile("" : "+v"(rv[u]), "+v"(sv[u]));
            const int64_t h = h0 + 256 * u;
            if (h < nint) {
                const int d = 63 - __clzll((unsigned long long)(h + 1));
                if (d != cd) {
                    if (cd >= 0 && cd < STATS_DEPTHS)
                        atomicMax(&smax[cd + 1], cm);
                    cd = d;
                    cm = 0;
                }
                cm = std::max(cm, rv[u]);
                mycap += (sv[u] == ACA_CAPPED) ? 1 : 0;
            }
        }
    }
    if (cd >= 0 && cd < STATS_DEPTHS)
        atomicMax(&smax[cd + 1], cm);
    for (int off = 32; off > 0; off >>= 1)
        mycap += __shfl_xor(mycap, off, 64);
    if ((threadIdx.x & 63) == 0)
        atomicAdd(&scap, mycap);
    __syncthreads();
    if (threadIdx.x < 48)
        rmax[threadIdx.x] = smax[threadIdx.x];
    if (threadIdx.x == 48)
        rmax[48] = scap;
    if (threadIdx.x == 49)
        rmax[49] = ndone ? *ndone : 0;
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

// 64 pinned ints per host thread, allocated on first use and released when
// the thread ends
int *pinned_scratch()
{
    struct Buf {
        int *p = nullptr;
        ~Buf()
        {
            if (p)
                (void)hipHostFree(p);
        }
    };
    thread_local Buf buf;
    if (!buf.p)
        HIP_TRY(hipHostMalloc((void **)&buf.p, 64 * sizeof(int), hipHostMallocDefault));
    return buf.p;
}

// Wait for the stream by polling an event recorded on it (one per host
// thread and device): the rank statistics sit on the likelihood's critical
// path, and a blocking synchronization wakes the thread tens of microseconds
// after the copies end.
void host_wait(hipStream_t s)
{
    struct Ev {
        hipEvent_t e[16] = {};
        ~Ev()
        {
            for (hipEvent_t x : e)
                if (x)
                    (void)hipEventDestroy(x);
        }
    };
    thread_local Ev ev;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 16) {
        HIP_TRY(hipStreamSynchronize(s));
        return;
    }
    if (!ev.e[dev])
        HIP_TRY(hipEventCreateWithFlags(&ev.e[dev], hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev.e[dev], s));
    for (;;) {
        const hipError_t q = hipEventQuery(ev.e[dev]);
        if (q == hipSuccess)
            break;
        if (q != hipErrorNotReady)
            HIP_TRY(q);
    }
}

// A growable pinned int buffer per host thread and slot (0: the per-node ranks
// read back after compression, 1: the column list uploaded before the
// leaves, 2: a speculative call's rank statistics, 3: values read back at
// the end of a call, the status word at int 8), so those copies go straight between
// device and host memory.  A slot is rewritten only after the stream has been
// synchronized since its last copy (each compression, and each read of the
// status, ends with a synchronization).
int *pinned_ints(size_t n, int slot)
{
    struct Buf {
        int *p[4] = {nullptr, nullptr, nullptr, nullptr};
        size_t cap[4] = {0, 0, 0, 0};
        ~Buf()
        {
            for (int i = 0; i < 4; ++i)
                if (p[i])
                    (void)hipHostFree(p[i]);
        }
    };
    thread_local Buf buf;
    if (buf.cap[slot] < n) {
        if (buf.p[slot])
            HIP_TRY(hipHostFree(buf.p[slot]));
        buf.p[slot] = nullptr;
        buf.cap[slot] = 0;
        const size_t want = std::max<size_t>(n, 4096);
        HIP_TRY(hipHostMalloc((void **)&buf.p[slot], want * sizeof(int), hipHostMallocDefault));
        buf.cap[slot] = want;
    }
    return buf.p[slot];
}

// rank statistics of all blocks and their copies to the host (one
// synchronization): rmax in pinned[0..L+1], the capped count in pinned[48],
// the finished large-block count (if d_ndone is given) in pinned[49]
static void read_rank_stats(Pipeline &P, const int *rank, const int *status, int *d_rmax,
                            int *d_capped, const int *d_ndone, int *pinned)
{
    const Plan &p = *P.plan;
    hipStream_t s = P.stream;
    (void)d_capped;   // the capped count travels in d_rmax[48]
    {
        ProfScope ps(s, PS_ACA_MISC);
        aca_stats_kernel<<<1, 256, 0, s>>>(rank, status, p.nint, d_rmax, d_ndone);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(pinned, d_rmax, sizeof(int) * 64, hipMemcpyDeviceToHost, s));
    int *hr = pinned_ints((size_t)p.nint, 0);
    HIP_TRY(hipMemcpyAsync(hr, rank, sizeof(int) * p.nint, hipMemcpyDeviceToHost, s));
    host_wait(s);
    std::memcpy(P.ranks.data(), hr, sizeof(int) * p.nint);
}

// After a speculative compression (no host wait): the rank statistics of
// aca_stats_kernel (rmax[j] = largest rank at depth j - 1, rmax[48] capped,
// rmax[49] converged large blocks) against the panel widths the call assumed
// (w, per depth index as rmax) and the large-block count.  The actual
// statistics are kept in save[0, 64) for the host.  On a miss (a rank above
// its width, or a large block still running) the status word records it and
// every block's rank is clamped to its depth's width, so that the rest of the
// pipeline stays inside its buffers; the call is then redone by the host.
// rmax[0 .. L+1] finally holds the assumed widths, as the padding kernel
// expects.
struct SpecArgs {
    int *rank;
    int64_t nint;
    int *rmax, *save;
    int *status;
    int active;   // large blocks that must have converged
    int L;
    int w[64];
    const int64_t *cofa;   // panel column offsets (device)
    int *cols;             // the column list the assumed widths give
};

__global__ __launch_bounds__(256) void spec_check_kernel(SpecArgs a)
{
    __shared__ int miss;
    if (threadIdx.x == 0)
        miss = (a.active > 0 && a.rmax[49] < a.active) ? 1 : 0;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int v = a.rmax[threadIdx.x];
        a.save[threadIdx.x] = v;
        if ((int)threadIdx.x <= a.L + 1 && v > a.w[threadIdx.x])
            miss = 1;   // every writer stores the same value
    }
    __syncthreads();
    if (miss) {
        for (int64_t h = threadIdx.x; h < a.nint; h += blockDim.x) {
            int d = 0;
            while (((int64_t)2 << d) - 1 <= h)
                ++d;
            a.rank[h] = min(a.rank[h], a.w[d + 1]);
        }
        if (threadIdx.x == 0)
            atomicOr(a.status, DS_SPEC_MISS);
    }
    if ((int)threadIdx.x <= a.L + 1 && threadIdx.x < 48)
        a.rmax[threadIdx.x] = a.w[threadIdx.x];
    // column list: 0, then depth j's panel columns cofa[j] .. cofa[j] + w[j] - 1
    // (the same list the host builds from the widths)
    __shared__ int start[64];
    if (threadIdx.x == 0) {
        int c = 1;
        for (int j = 1; j <= a.L; ++j) {
            start[j] = c;
            c += a.w[j];
        }
        a.cols[0] = 0;
    }
    __syncthreads();
    for (int j = 1; j <= a.L; ++j)
        for (int c = threadIdx.x; c < a.w[j]; c += blockDim.x)
            a.cols[start[j] + c] = (int)(a.cofa[j] + c);
}

// Per-call initialization in one launch instead of a memset or copy each:
// zero the status words, the counters and every block's rank and state, and
// write the panel column offsets (passed by value).
struct InitArgs {
    int *status;   // 4 status words
    int *ndone, *capped;
    int *rank, *astatus;
    int64_t nint;
    int64_t *cofa;
    int ncofa;
    int64_t cofa_v[64];
};

__global__ __launch_bounds__(256) void pipeline_init_kernel(InitArgs a)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = g; i < a.nint; i += (int64_t)gridDim.x * blockDim.x) {
        a.rank[i] = 0;   // blocks with an empty side keep rank 0 and count as done
        a.astatus[i] = 0;
    }
    if (blockIdx.x == 0) {
        if (threadIdx.x < 4)
            a.status[threadIdx.x] = 0;
        if (threadIdx.x == 0 && a.ndone) {
            *a.ndone = 0;
            *a.capped = 0;
        }
        if ((int)threadIdx.x < a.ncofa)
            a.cofa[threadIdx.x] = a.cofa_v[threadIdx.x];
    }
}

// A second stream of the calling host thread on each device (default
// priority), with the events that fork work onto it and join it back.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

static SideStream &side_stream()
{
    struct Table {
        SideStream e[16];
        ~Table()
        {
            for (SideStream &x : e) {
                if (x.s)
                    (void)hipStreamDestroy(x.s);
                if (x.fork)
                    (void)hipEventDestroy(x.fork);
                if (x.join)
                    (void)hipEventDestroy(x.join);
            }
        }
    };
    thread_local Table t;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 16)
        throw Error{HODLR_EDEVICE, "device index above 15"};
    SideStream &x = t.e[dev];
    if (!x.s) {
        HIP_TRY(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&x.fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&x.join, hipEventDisableTiming));
    }
    return x;
}

// Makes the pipeline's stream wait for what was forked onto the side stream,
// at the latest when it goes out of scope (also when an error unwinds).
struct SideJoin {
    hipStream_t main;
    SideStream *side = nullptr;
    void wait()
    {
        if (side) {
            SideStream *x = side;
            side = nullptr;
            HIP_TRY(hipStreamWaitEvent(main, x->join, 0));
        }
    }
    ~SideJoin()
    {
        if (side)
            (void)hipStreamWaitEvent(main, side->join, 0);
    }
};

// one pass over the large blocks' chunks, specialized on the chunk length and
// on the rank bound of the LDS arrays
template <bool ROW>
static void big_pass(const Plan &p, int nchunk, hipStream_t s, const BigArgs &B)
{
    constexpr int E1 = ACA_CHUNK_1D / ACA_THREADS, EN = ACA_CHUNK_ND / ACA_THREADS;
    const bool narrow = p.cap <= RMAX_LDS;
    if (p.aca_chunk == ACA_CHUNK_1D) {
        if (narrow)
            aca_big_pass_kernel<ROW, E1, RMAX_LDS><<<nchunk, ACA_THREADS, 0, s>>>(B);
        else
            aca_big_pass_kernel<ROW, E1, RMAX_ABS><<<nchunk, ACA_THREADS, 0, s>>>(B);
    } else {
        if (narrow)
            aca_big_pass_kernel<ROW, EN, RMAX_LDS><<<nchunk, ACA_THREADS, 0, s>>>(B);
        else
            aca_big_pass_kernel<ROW, EN, RMAX_ABS><<<nchunk, ACA_THREADS, 0, s>>>(B);
    }
}

void run_sketch_levels(Pipeline &P, int *rank, int *status);   // sketch.hip

// The compression stage: adaptive cross approximation, or (plans made with
// HODLR_COMPRESS_SKETCH) the randomized sketch; both end with the rank
// statistics on the host and the panels' padding columns zeroed.
void run_aca(Pipeline &P)
{
    const Plan &p = *P.plan;
    hipStream_t s = P.stream;
    P.rmax.assign(p.L + 2, 0);
    P.ranks.assign(p.nint, 0);
    P.capped = 0;
    InitArgs ia{};
    ia.status = wsp<int>(P, P.lay.status);
    if (p.L == 0) {
        pipeline_init_kernel<<<1, 256, 0, s>>>(ia);
        HIP_TRY(hipGetLastError());
        return;
    }
    int *pinned = P.host_ints ? P.host_ints : pinned_scratch();
    int64_t *d_cofa = wsp<int64_t>(P, P.lay.misc);          // [0, 512): column offsets
    int *d_rmax = wsp<int>(P, P.lay.misc + 512);             // [512, 784): rmax per depth
    int *d_capped = wsp<int>(P, P.lay.misc + 784);
    int *d_ndone = wsp<int>(P, P.lay.misc + 1024);
    if (p.cofa.size() > 64)
        throw Error{HODLR_EINVAL, "more than 62 tree levels"};
    AcaArgs A;
    A.x = P.x;
    A.n = p.n;
    A.kp = P.kp;
    A.tol = P.tol;
    A.W = wsp<double>(P, P.lay.W);
    A.start = p.d_start;
    A.end = p.d_end;
    A.cofa = d_cofa;
    A.cap = p.cap;
    int *rank = wsp<int>(P, P.lay.rank);
    int *status = wsp<int>(P, P.lay.aca_status);
    ia.ndone = d_ndone;
    ia.capped = d_capped;
    ia.rank = rank;
    ia.astatus = status;
    ia.nint = p.nint;
    ia.cofa = d_cofa;
    ia.ncofa = (int)p.cofa.size();
    for (size_t j = 0; j < p.cofa.size(); ++j)
        ia.cofa_v[j] = p.cofa[j];
    {
        ProfScope ps(s, PS_ACA_MISC);
        const int64_t nb = std::min<int64_t>((p.nint + 255) / 256, 1024);
        pipeline_init_kernel<<<(unsigned)std::max<int64_t>(nb, 1), 256, 0, s>>>(ia);
    }
    HIP_TRY(hipGetLastError());
    // speculation: the previous call's widths and large-block step count
    const int hint = __atomic_load_n(&p.aca_iters, __ATOMIC_RELAXED);
    const bool spec = P.spec && (int)P.spec->size() == p.L + 2 && p.L + 2 <= 48 &&
                      p.compressor == HODLR_COMPRESS_ACA && (p.aca_big.empty() || hint > 0);
    P.spec_run = spec;
    if (p.compressor == HODLR_COMPRESS_SKETCH) {
        run_sketch_levels(P, rank, status);
        read_rank_stats(P, rank, status, d_rmax, d_capped, nullptr, pinned);
        for (int j = 0; j <= p.L + 1 && j < 48; ++j)
            P.rmax[j] = pinned[j];
        P.capped = pinned[48];
        ProfScope ps(s, PS_ACA_MISC);
        if (!p.pad_chunks.empty())
            aca_pad_kernel<<<(unsigned)p.pad_chunks.size(), 256, 0, s>>>(A.W, p.n, p.d_pad_chunks,
                                                                          rank, d_rmax, d_cofa);
        HIP_TRY(hipGetLastError());
        return;
    }
    const int nbig = (int)p.aca_big.size();
    // small blocks: the whole loop per work-group.  When there are large
    // blocks too, they run on the side stream, alongside the large blocks'
    // passes (which occupy few work-groups per launch), and are joined before
    // the first rank statistics.
    SideJoin join{s};
    if (!p.aca_small.empty()) {
        hipStream_t ss = s;
        if (nbig > 0 && P.side_stream) {
            SideStream &x = side_stream();
            HIP_TRY(hipEventRecord(x.fork, s));
            HIP_TRY(hipStreamWaitEvent(x.s, x.fork, 0));
            ss = x.s;
        }
        SmallArgs S;
        S.a = A;
        S.nodes = p.d_aca_small;
        S.rank = rank;
        S.status = status;
        {
            ProfScope ps(ss, PS_ACA_SMALL);
            // blocks with both sides <= ACA_TINY (listed last) run on one wave,
            // with wave-level reductions only
            const int nwide = p.aca_small_wide;
            const bool narrow = p.cap <= RMAX_LDS;
            if (nwide > 0) {
                if (narrow)
                    aca_small_kernel<ACA_SMALL_TH, ACA_SMALL, RMAX_LDS>
                        <<<(unsigned)nwide, ACA_SMALL_TH, 0, ss>>>(S);
                else
                    aca_small_kernel<ACA_SMALL_TH, ACA_SMALL, RMAX_ABS>
                        <<<(unsigned)nwide, ACA_SMALL_TH, 0, ss>>>(S);
                HIP_TRY(hipGetLastError());
            }
            const int ntiny = (int)p.aca_small.size() - nwide;
            if (ntiny > 0) {
                S.nodes = p.d_aca_small + nwide;
                if (narrow)
                    aca_small_kernel<64, ACA_TINY, RMAX_LDS><<<(unsigned)ntiny, 64, 0, ss>>>(S);
                else
                    aca_small_kernel<64, ACA_TINY, RMAX_ABS><<<(unsigned)ntiny, 64, 0, ss>>>(S);
                HIP_TRY(hipGetLastError());
            }
        }
        if (ss != s) {
            SideStream &x = side_stream();
            HIP_TRY(hipEventRecord(x.join, ss));
            join.side = &x;
        }
    }
    if (nbig > 0) {
        BigState *st0 = wsp<BigState>(P, P.lay.aca_state);
        BigState *st1 = st0 + nbig;
        double *rrec = wsp<double>(P, P.lay.aca_part);
        double *crec = rrec + (int64_t)p.aca_row.size() * p.aca_pw;
        {
            ProfScope ps(s, PS_ACA_MISC);
            aca_big_init_kernel<<<(nbig + 255) / 256, 256, 0, s>>>(st0, p.d_aca_big, nbig, A);
        }
        BigArgs R, C;
        R.a = C.a = A;
        R.bnode = C.bnode = p.d_aca_big;
        R.pw = C.pw = p.aca_pw;
        R.used = C.used = wsp<int>(P, P.lay.aca_used);
        R.vdots = C.vdots = wsp<double>(P, P.lay.aca_vdots);
        R.ndone = C.ndone = d_ndone;
        R.chunks = p.d_aca_row;   // rows of beta
        R.cidx = p.d_aca_rowidx;
        R.pnch = p.d_aca_ncol;    // previous pass = column records
        R.pbase = p.d_aca_colbase;
        R.sin = st0;
        R.sout = st1;
        R.pin = crec;
        R.pout = rrec;
        C.chunks = p.d_aca_col;   // rows of alpha
        C.cidx = p.d_aca_colidx;
        C.pnch = p.d_aca_nrow;
        C.pbase = p.d_aca_rowbase;
        C.sin = st1;
        C.sout = st0;
        C.pin = rrec;
        C.pout = crec;
        const int nrow = (int)p.aca_row.size(), ncol = (int)p.aca_col.size();
        const int max_iter = (p.cap + 1) * (ZERO_RETRY + 2) + 4;
        int it = 0;
        for (; it < max_iter; ++it) {
            {
                ProfScope ps(s, PS_ACA_ROW);
                big_pass<true>(p, nrow, s, R);
            }
            {
                ProfScope ps(s, PS_ACA_COL);
                big_pass<false>(p, ncol, s, C);
            }
            HIP_TRY(hipGetLastError());
            if (spec) {
                // the previous call's step count, no poll: the device check
                // below tells whether every block converged
                if (it + 1 < hint)
                    continue;
                join.wait();
                ProfScope ps(s, PS_ACA_MISC);
                aca_big_finish_kernel<<<(nbig + 255) / 256, 256, 0, s>>>(st0, p.d_aca_big, nbig, rank,
                                                                         status);
                break;
            }
            // A converged block is counted by the row pass that absorbs its last
            // column.  Poll from the step where the previous call on this plan
            // finished (else every other step from the third on); a poll that
            // may be the last also takes the ranks and their statistics, so
            // that one synchronization serves both.  If blocks remain, the
            // loop goes on and the final poll rewrites them.
            const bool poll = hint > 0 ? it + 1 >= hint : (it >= 2 && (it & 1) == 0);
            if (poll) {
                join.wait();   // the small blocks' ranks are part of the statistics
                {
                    ProfScope ps(s, PS_ACA_MISC);
                    aca_big_finish_kernel<<<(nbig + 255) / 256, 256, 0, s>>>(st0, p.d_aca_big,
                                                                             nbig, rank, status);
                }
                read_rank_stats(P, rank, status, d_rmax, d_capped, d_ndone, pinned);
                if (pinned[49] >= p.aca_big_active)
                    break;
            }
        }
        if (it >= max_iter)
            throw Error{HODLR_EDEVICE, "cross approximation did not terminate"};
        if (!spec)
            __atomic_store_n(&p.aca_iters, it + 1, __ATOMIC_RELAXED);
    } else if (!spec) {
        read_rank_stats(P, rank, status, d_rmax, d_capped, nullptr, pinned);
    }
    if (spec) {
        join.wait();
        SpecArgs sa{};
        sa.rank = rank;
        sa.nint = p.nint;
        sa.rmax = d_rmax;
        sa.save = wsp<int>(P, P.lay.misc + MISC_SPEC);
        sa.status = wsp<int>(P, P.lay.status);
        sa.active = nbig > 0 ? p.aca_big_active : 0;
        sa.L = p.L;
        for (int j = 0; j <= p.L + 1; ++j)
            sa.w[j] = (*P.spec)[j];
        sa.cofa = d_cofa;
        sa.cols = wsp<int>(P, P.lay.cols);
        {
            ProfScope ps(s, PS_ACA_MISC);
            aca_stats_kernel<<<1, 256, 0, s>>>(rank, status, p.nint, d_rmax, nbig > 0 ? d_ndone : nullptr);
            spec_check_kernel<<<1, 256, 0, s>>>(sa);
        }
        HIP_TRY(hipGetLastError());
        P.rmax.assign(P.spec->begin(), P.spec->end());
        P.capped = 0;   // read with the call's status
    } else {
        for (int j = 0; j <= p.L + 1 && j < 48; ++j)
            P.rmax[j] = pinned[j];
        P.capped = pinned[48];
    }
    // zero the padding columns of every block below its panel's maximum rank
    ProfScope ps(s, PS_ACA_MISC);
    if (!p.pad_chunks.empty())
        aca_pad_kernel<<<(unsigned)p.pad_chunks.size(), 256, 0, s>>>(A.W, p.n, p.d_pad_chunks,
                                                                      rank, d_rmax, d_cofa);
    HIP_TRY(hipGetLastError());
}

}  // namespace hodlr
