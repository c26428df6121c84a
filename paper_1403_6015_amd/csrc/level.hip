// Level stage: factor the block-diagonal low-rank updates of the identity
// level by level from the leaves' parents to the root (§3.2).
//
// For a node tau with children alpha, beta and bases W (K(alpha,beta) ~
// W_alpha W_beta^T), once the finer inverses are applied the diagonal block
// of tau is diag(C_alpha, C_beta) (I + diag(W~_alpha, W~_beta) R) with
// R = [[0, W_beta^T], [W_alpha^T, 0]] (the block low-rank update form of
// §3.2).  Sherman-Morrison-Woodbury turns its inverse into the small coupling
// matrix M = I + R diag(W~_alpha, W~_beta) = [[I, P], [Q, I]] with
// P = W_beta^T W~_beta and Q = W_alpha^T W~_alpha, and Sylvester's theorem
// (§4) gives det of the block as det M = det(I - Q P).
//
// Per level three launches (four when the top levels' partial sums are
// large):
//   reduce  -- T = [W_beta^T X_beta; W_alpha^T X_alpha] over every column X
//              still to be updated plus the child panel itself (which yields
//              P and Q), as per-chunk partial sums: for ranks up to 8 one wave
//              per chunk with W's rows in registers (bandwidth-bound), above
//              that on FP64 MFMA;
//   solve   -- one work-group per node sums the partials (or a sum kernel
//              with one thread per output does it first), forms I - Q P,
//              LU-factors it with partial pivoting in LDS, records its
//              log-det, and solves M S = T for the remaining columns
//              (s2 = (I - QP)^{-1} (t2 - Q t1), s1 = t1 - P s2);
//   update  -- X_alpha -= W~_alpha S_top, X_beta -= W~_beta S_bottom (one
//              thread per row for small ranks, FP64 MFMA above 8).
// The solve path reuses the three kernels on the single vector z with the
// stored small factors.
#include "common.h"

namespace hodlr {

constexpr int LV_THREADS = 256;
constexpr int LV_CB = 32;    // right-hand sides per batch in the node solve
// threads per node in the node solve (n = 2^20: 256 threads 0.37 ms per
// likelihood, one wave 0.81 ms)
constexpr int LV_SOLVE_TH = 256;
// levels whose nodes each hold more than LV_SUM_MIN record entries (chunks
// per node x 2 r x columns) sum them in a kernel of their own, one thread per
// output, before the node solves.  2-D SE at n = 2^18 (ranks up to 64): node
// solves 8.25 -> 5.0 ms per likelihood; doing so on every level with at most
// 64 nodes cost the 1-D Matern workload 0.08 ms (small records, one more
// launch per level).
constexpr double LV_SUM_MIN = 262144.0;
// levels with at most LV_SPLIT_NODES nodes and more than LV_SPLIT_COLS
// columns to update also sum first, so that their node solves can split the
// column batches over several work-groups per node (at most LV_SPLIT_GROUPS
// work-groups per node, LV_SPLIT_TOTAL in all).  2-D SE at n = 2^18: node
// solves 3.2 ms with the split on levels of at most 64 nodes, 2.2 ms up to
// 256 nodes, 2.1 ms up to 1024; the 1-D Matern panels (at most 42 columns)
// never reach LV_SPLIT_COLS.
constexpr unsigned LV_SPLIT_NODES = 1024;
constexpr int LV_SPLIT_COLS = 4 * LV_CB;
constexpr unsigned LV_SPLIT_GROUPS = 16;
constexpr unsigned LV_SPLIT_TOTAL = 4096;

struct LevelArgs {
    int64_t n;
    const double *W;   // compressed bases
    void *Xt;          // applied bases: double, or float in the mixed form
    const int *cols;
    int ncnt;          // columns entering the reduction (prefix of cols)
    int nrhs;          // columns updated (prefix of cols)
    int64_t colW;      // first column of the child panel
    int rstride;       // reserved rank of the child panel at run time
    const int *rank;
    const Chunk *chunks;
    const int *nch, *base;
    int64_t node0;
    double *part;
    double *Tbuf, *Sbuf;
    int64_t tstride;
    double *small;
    int64_t sstride;
    double *node_ld;
    int *status;
    int factor;        // 1: build the coupling factors; 0: apply stored ones
    int cgrp;          // columns per work-group of the small-rank reduction
    int rows;          // rows per chunk (a node's chunks: its alpha rows, then its beta rows)
    int tsum;          // 1: T was summed from the records by level_sum_kernel
    // records written by the fused pass of the level below (nullable): node
    // loc's alpha records are the chunks of its alpha child in that level's
    // table ([cbase[2 loc], + cnch[2 loc])), its beta records those of its beta
    // child, right after them
    const int *cbase, *cnch;
    // the fused pass (update of this level, records of the level above):
    // that level's panel column, rank stride and record columns (= nrhs)
    int64_t colWp;
    int rstride_p;
    BatchArgs B;
};

// a node's record ranges: alpha [base, base + na), beta [base + na, base + nch)
__device__ __forceinline__ void node_records(const LevelArgs &A, int64_t loc, int &base, int &na,
                                             int &nch)
{
    if (A.cbase) {
        base = A.cbase[2 * loc];
        na = A.cnch[2 * loc];
        nch = na + A.cnch[2 * loc + 1];
        return;
    }
    nch = A.nch[loc];
    base = A.base[loc];
    const int64_t ns = A.chunks[base].lo, ne = A.chunks[base + nch - 1].hi;
    const int64_t alen = (ne - ns) / 2;
    na = (int)((alen + A.rows - 1) / A.rows);
}

// this work-group's batch item: offset every per-item pointer
__device__ __forceinline__ LevelArgs item_args(LevelArgs A)
{
    const int it = blockIdx.z;
    if (it) {
        A.W = ioff(A.W, A.B, it);
        A.Xt = ioff(A.Xt, A.B, it);
        A.rank = ioff(A.rank, A.B, it);
        A.part = ioff(A.part, A.B, it);
        A.Tbuf = ioff(A.Tbuf, A.B, it);
        A.Sbuf = ioff(A.Sbuf, A.B, it);
        A.small = ioff(A.small, A.B, it);
        A.node_ld = ioff(A.node_ld, A.B, it);
        A.status = ioff(A.status, A.B, it);
    }
    return A;
}

// Small-rank variants (panel rank <= R, the usual case for 1-D kernels):
// one wave per chunk for the reduction, the chunk's W rows kept in registers
// and every column reduced across the wave; one thread per row for the
// update, with S in LDS.  Both stream each X column once, coalesced.
// columns per work-group of the small-rank reduction: the plan's red_grp (8 or
// 64).  Every work-group of a chunk re-reads the chunk's W rows, so wide groups
// read W once; narrow groups give more work-groups.

// Body of the small-rank reduction for one chunk (SR rows per lane, chunk =
// 64 SR rows; CU columns per iteration).  Row of slot t of a lane: lo + lane
// + 64 t, or with PAIR lo + 128 (t / 2) + 2 lane + t % 2, so that an FP32
// panel is read as float2 (two adjacent rows per lane: as many bytes per load
// instruction as the FP64 panel, which keeps twice the bytes in flight).
template <typename PT, int R, int SR, int CU, bool PAIR>
__device__ __forceinline__ void reduce_chunk(const LevelArgs &A, const Chunk &ch, int r, double *red)
{
    const double *__restrict__ Wp = A.W;
    const PT *__restrict__ Xp = (const PT *)A.Xt;
    const int lane = threadIdx.x;
    const int64_t n = A.n;
    auto row = [&](int t) -> int64_t {
        return PAIR ? ch.lo + 128 * (t >> 1) + 2 * lane + (t & 1) : ch.lo + lane + 64 * t;
    };
    double w[SR][R];
    bool ok[SR];
#pragma unroll
    for (int t = 0; t < SR; ++t) {
        const int64_t i = row(t);
        ok[t] = i < ch.hi;
#pragma unroll
        for (int l = 0; l < R; ++l)
            w[t][l] = (ok[t] && l < r) ? Wp[(A.colW + l) * n + i] : 0.0;
    }
    double *rec = A.part + (int64_t)ch.part * A.rstride * A.ncnt;
    const int cend = min(A.ncnt, (int)(blockIdx.y + 1) * A.cgrp);
    for (int c0 = blockIdx.y * A.cgrp; c0 < cend; c0 += CU) {
        const PT *xc[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u)
            xc[u] = (c0 + u < cend) ? Xp + (int64_t)A.cols[c0 + u] * n : nullptr;
        double acc[CU][R];
#pragma unroll
        for (int u = 0; u < CU; ++u)
#pragma unroll
            for (int l = 0; l < R; ++l)
                acc[u][l] = 0.0;
        if constexpr (PAIR) {
            static_assert(SR % 2 == 0, "pairs of slots");
#pragma unroll
            for (int p = 0; p < SR / 2; ++p) {
                if (ok[2 * p]) {
#pragma unroll
                    for (int u = 0; u < CU; ++u) {
                        double x0 = 0.0, x1 = 0.0;
                        if (xc[u]) {
                            const int64_t i0 = row(2 * p);
                            if (ok[2 * p + 1]) {
                                const float2 v = *(const float2 *)(xc[u] + i0);
                                x0 = v.x;
                                x1 = v.y;
                            } else {
                                x0 = xc[u][i0];
                            }
                        }
#pragma unroll
                        for (int l = 0; l < R; ++l)
                            acc[u][l] += w[2 * p][l] * x0 + w[2 * p + 1][l] * x1;
                    }
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < SR; ++t) {
                if (ok[t]) {
#pragma unroll
                    for (int u = 0; u < CU; ++u) {
                        const double x = xc[u] ? (double)xc[u][row(t)] : 0.0;
#pragma unroll
                        for (int l = 0; l < R; ++l)
                            acc[u][l] += w[t][l] * x;
                    }
                }
            }
        }
        // cross-lane sums of the CU*R accumulators through LDS: each output
        // gets 64/(CU*R) lanes (or one lane several outputs), then a few
        // shuffles, instead of one full wave reduction per output
        constexpr int NO = CU * R;
#pragma unroll
        for (int u = 0; u < CU; ++u)
#pragma unroll
            for (int l = 0; l < R; ++l)
                red[lane * (NO + 1) + u * R + l] = acc[u][l];
        __syncthreads();
        if constexpr (NO <= 64) {
            constexpr int G = 64 / NO;            // lanes per output (power of two)
            const int o = lane / G, sub = lane % G;
            double a = 0.0;
            for (int q = sub; q < 64; q += G)
                a += red[q * (NO + 1) + o];
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1)
                a += __shfl_xor(a, off, 64);
            const int u = o / R, l = o % R;
            if (sub == 0 && l < r && c0 + u < cend)
                rec[(int64_t)l * A.ncnt + c0 + u] = a;
        } else {
            for (int o = lane; o < NO; o += 64) {
                double a = 0.0;
                for (int q = 0; q < 64; ++q)
                    a += red[q * (NO + 1) + o];
                const int u = o / R, l = o % R;
                if (l < r && c0 + u < cend)
                    rec[(int64_t)l * A.ncnt + c0 + u] = a;
            }
        }
        __syncthreads();
    }
}


// SR rows per lane (chunk = 64 SR rows), CU columns per iteration
template <typename PT, int R, int SR, int CU>
__global__ __launch_bounds__(64) void level_reduce_small_kernel(LevelArgs A0)
{
    const LevelArgs A = item_args(A0);
    const Chunk ch = A.chunks[blockIdx.x];
    const int r = A.rank[ch.node];
    if (r == 0)
        return;
    constexpr int NO = CU * R;
    __shared__ double red[64 * (NO + 1)];
    // an FP32 panel with an even chunk start (and even n) is read in pairs
    if constexpr (sizeof(PT) == 4 && SR % 2 == 0) {
        if (((ch.lo | A.n) & 1) == 0) {
            reduce_chunk<PT, R, SR, CU, true>(A, ch, r, red);
            return;
        }
    }
    reduce_chunk<PT, R, SR, CU, false>(A, ch, r, red);
}

template <typename PT, int R>
__global__ __launch_bounds__(LV_THREADS) void level_update_small_kernel(LevelArgs A0, int smax)
{
    const LevelArgs A = item_args(A0);
    PT *__restrict__ Xp = (PT *)A.Xt;
    extern __shared__ double sS[];   // R x nrhs
    const Chunk ch = A.chunks[blockIdx.x];
    const int r = A.rank[ch.node];
    if (r == 0)
        return;
    const int64_t n = A.n;
    const int64_t loc = ch.node - A.node0;
    const double *S = A.Sbuf + loc * A.tstride;
    const int rowoff = ch.side ? A.rstride : 0;   // alpha uses S_top, beta S_bottom
    const int nrhs = A.nrhs;
    for (int idx = threadIdx.x; idx < R * nrhs; idx += LV_THREADS) {
        int l = idx / nrhs, c = idx % nrhs;
        sS[idx] = (l < r) ? S[(int64_t)(rowoff + l) * nrhs + c] : 0.0;
    }
    __syncthreads();
    for (int64_t i = ch.lo + threadIdx.x; i < ch.hi; i += LV_THREADS) {
        double w[R];
#pragma unroll
        for (int l = 0; l < R; ++l)
            w[l] = (l < r) ? (double)Xp[(A.colW + l) * n + i] : 0.0;
        for (int c = 0; c < nrhs; ++c) {
            PT *px = Xp + (int64_t)A.cols[c] * n + i;
            double a = *px;
#pragma unroll
            for (int l = 0; l < R; ++l)
                a -= w[l] * sS[l * nrhs + c];
            *px = (PT)a;
        }
    }
}

// Cross-lane moves for the butterfly sums of the fused pass (values in
// registers, no LDS): DPP within a row of 16 lanes, the lane-swap
// instructions across rows and across the two halves of the wave.
template <int CTRL>
__device__ __forceinline__ double dpp64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// lanes L and L ^ M (M = 32 or 16): L with bit M clear returns a(L) +
// a(L ^ M), L with the bit set b(L) + b(L ^ M)
template <int M>
__device__ __forceinline__ double swap_sum(double a, double b)
{
    const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
    unsigned lo0 = (unsigned)x, hi0 = (unsigned)(x >> 32), lo1 = (unsigned)y, hi1 = (unsigned)(y >> 32);
    if constexpr (M == 32) {
        const auto l = __builtin_amdgcn_permlane32_swap(lo0, lo1, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi0, hi1, false, false);
        lo0 = l[0], lo1 = l[1], hi0 = h[0], hi1 = h[1];
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(lo0, lo1, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi0, hi1, false, false);
        lo0 = l[0], lo1 = l[1], hi0 = h[0], hi1 = h[1];
    }
    return __longlong_as_double(((long long)hi0 << 32) | lo0) +
           __longlong_as_double(((long long)hi1 << 32) | lo1);
}

// DPP patterns pairing each lane with one whose bit M differs (M <= 8):
// row mirror (i <-> 15 - i), half-row mirror (i <-> 7 - i), quad swaps
template <int M>
__device__ __forceinline__ double pair_move(double v)
{
    if constexpr (M == 8)
        return dpp64<0x140>(v);
    else if constexpr (M == 4)
        return dpp64<0x141>(v);
    else if constexpr (M == 2)
        return dpp64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    else
        return dpp64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
}

// One halving step of the butterfly over v[0, 2H): the pairing of step M
// joins lanes that hold the same outputs and disjoint sets of summed lanes;
// a lane keeps the upper half if its bit M is set.
template <int M, int H>
__device__ __forceinline__ void halve(double *v, int lane)
{
    if constexpr (M >= 16) {
#pragma unroll
        for (int j = 0; j < H; ++j)
            v[j] = swap_sum<M>(v[j], v[j + H]);
    } else {
        const bool up = (lane & M) != 0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const double send = up ? v[j] : v[j + H];
            const double keep = up ? v[j + H] : v[j];
            v[j] = keep + pair_move<M>(send);
        }
    }
}

// sums of NO values per lane over the 64 lanes: afterwards v[0] of lane l is
// output l / (64 / NO), complete in every lane
template <int NO>
__device__ __forceinline__ double wave_sums(double *v, int lane)
{
    static_assert(NO == 16 || NO == 32, "outputs per wave");
    halve<32, NO / 2>(v, lane);
    halve<16, NO / 4>(v, lane);
    halve<8, NO / 8>(v, lane);
    halve<4, NO / 16>(v, lane);
    if constexpr (NO == 32)
        halve<2, 1>(v, lane);
    double a = v[0];
    // the lanes sharing an output: a quad (NO = 16) or a pair (NO = 32)
    if constexpr (NO == 16)
        a += pair_move<2>(a);
    a += pair_move<1>(a);
    return a;
}

// Fused pass for small ranks: the update of level d (X -= W~ S on the
// chunk's rows) and the reduction records of level d-1 on the same rows
// (W_{d-1}^T X over the chunk, of the updated X as stored), so that X is read
// once for both.  The columns updated at level d are exactly those level d-1
// reduces (its child panel is level d's last updated panel).  One work-group
// per level-d chunk, as many waves as the level's longest chunk needs (at
// most 8), RW rows per lane (row lo + 64 RW w + lane + 64 t of wave w; lanes
// past the chunk read its last row and contribute nothing), CU columns at a
// time with the next group's loads issued before this group's arithmetic.
// A group's CU x RP products are summed across the wave in registers
// (wave_sums) and left in LDS per wave and group; after the last group one
// barrier, then the work-group sums the waves.  The record of chunk q holds
// level d-1's rows l < rank(parent) at A.part + q rstride_p nrhs; the level
// above finds a node's records through its children's chunk ranges.
constexpr int LVF_MAXW = 8;
constexpr int LVF_CU = 4;

//
// With UPD false the same pass only reduces, for the level's own records
// (the deepest level, whose reduction no finer update can carry): no update,
// W of the chunk's own node against the A.ncnt reduced columns, records laid
// out as the small-rank reduction's.
template <typename PT, int R, int RP, int RW, bool UPD>
__global__ __launch_bounds__(64 * LVF_MAXW) void level_fused_kernel(LevelArgs A0)
{
    constexpr int CU = LVF_CU;
    constexpr int RU = UPD ? R : 1;   // update ranks held (none without the update)
    const LevelArgs A = item_args(A0);
    PT *__restrict__ Xp = (PT *)A.Xt;
    const double *__restrict__ Wp = A.W;
    const Chunk ch = A.chunks[blockIdx.x];
    const int r = UPD ? A.rank[ch.node] : 0;
    const int rp = UPD ? A.rank[(ch.node - 1) / 2] : A.rank[ch.node];
    if (r == 0 && rp == 0)
        return;
    const int64_t n = A.n;
    const int nrhs = UPD ? A.nrhs : A.ncnt;   // columns updated and reduced
    const int64_t colp = UPD ? A.colWp : A.colW;
    const int rsp = UPD ? A.rstride_p : A.rstride;
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
    constexpr int NO = CU * RP;
    constexpr int G = 64 / NO;   // lanes holding each output after the butterfly
    const int ngrp = (nrhs + CU - 1) / CU;
    extern __shared__ double sdyn[];
    double *sS = sdyn;                                 // R x nrhs (with the update)
    double *wsum = sdyn + (UPD ? R * nrhs : 0);        // [group][wave][NO]: the waves' sums
    int *scol = (int *)(wsum + (int64_t)ngrp * nw * NO);   // the column list
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x)
        scol[c] = A.cols[c];
    const int64_t loc = ch.node - A.node0;
    const double *S = A.Sbuf + loc * A.tstride;
    const int rowoff = ch.side ? A.rstride : 0;   // alpha uses S_top, beta S_bottom
    if (UPD) {
        for (int idx = threadIdx.x; idx < R * nrhs; idx += blockDim.x) {
            const int l = idx / nrhs, c = idx % nrhs;
            sS[idx] = (l < r) ? S[(int64_t)(rowoff + l) * nrhs + c] : 0.0;
        }
    }
    int64_t rowi[RW];
    bool ok[RW];
#pragma unroll
    for (int t = 0; t < RW; ++t) {
        const int64_t i = ch.lo + 64 * RW * wid + lane + 64 * t;
        ok[t] = i < ch.hi;
        rowi[t] = ok[t] ? i : ch.hi - 1;
    }
    // panel columns past a node's rank are read at its last column (or the
    // panel's first) and zeroed.  Every load is issued before the first
    // value is pinned in a register (the empty asm), so that the zeroing
    // selects do not turn into one branch and one wait per load.
    double wt[RW][RU], wp[RW][RP];
#pragma unroll
    for (int l = 0; l < RU; ++l) {
        const int64_t col = A.colW + (l < r ? l : (r > 0 ? r - 1 : 0));
#pragma unroll
        for (int t = 0; t < RW; ++t)
            wt[t][l] = UPD ? (double)Xp[col * n + rowi[t]] : 0.0;
    }
#pragma unroll
    for (int l = 0; l < RP; ++l) {
        const int64_t col = colp + (l < rp ? l : (rp > 0 ? rp - 1 : 0));
#pragma unroll
        for (int t = 0; t < RW; ++t)
            wp[t][l] = Wp[col * n + rowi[t]];
    }
#pragma unroll
    for (int t = 0; t < RW; ++t) {
#pragma unroll
        for (int l = 0; l < RU; ++l) {
            asm volatile("" : "+v"(wt[t][l]));
            wt[t][l] = (ok[t] && l < r) ? wt[t][l] : 0.0;
        }
#pragma unroll
        for (int l = 0; l < RP; ++l) {
            asm volatile("" : "+v"(wp[t][l]));
            wp[t][l] = (ok[t] && l < rp) ? wp[t][l] : 0.0;
        }
    }
    auto load = [&](int c0, PT *xc[CU], PT x[RW][CU]) {
#pragma unroll
        for (int u = 0; u < CU; ++u)
            xc[u] = Xp + (int64_t)scol[c0 + u < nrhs ? c0 + u : nrhs - 1] * n;
#pragma unroll
        for (int t = 0; t < RW; ++t)
#pragma unroll
            for (int u = 0; u < CU; ++u)
                x[t][u] = xc[u][rowi[t]];
    };
    __syncthreads();   // S and the column list staged
    PT *xc[CU], *xcn[CU];
    PT x[RW][CU], xn[RW][CU];
    if (ngrp > 0)
        load(0, xc, x);
    for (int g = 0; g < ngrp; ++g) {
        const int c0 = g * CU;
        if (g + 1 < ngrp)
            load(c0 + CU, xcn, xn);
        double v[NO];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            double sv[RU];
#pragma unroll
            for (int l = 0; l < RU; ++l)
                sv[l] = UPD && c0 + u < nrhs ? sS[l * nrhs + c0 + u] : 0.0;
#pragma unroll
            for (int l = 0; l < RP; ++l)
                v[u * RP + l] = 0.0;
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                double xs = (double)x[t][u];
                if constexpr (UPD) {
                    double a = xs;
#pragma unroll
                    for (int l = 0; l < R; ++l)
                        a -= wt[t][l] * sv[l];
                    const PT st = (PT)a;
                    if (r > 0 && ok[t] && c0 + u < nrhs)
                        xc[u][rowi[t]] = st;
                    xs = (double)st;
                }
#pragma unroll
                for (int l = 0; l < RP; ++l)
                    v[u * RP + l] += wp[t][l] * xs;
            }
        }
        if (rp > 0) {
            const double a = wave_sums<NO>(v, lane);
            if ((lane % G) == 0)
                wsum[((int64_t)g * nw + wid) * NO + lane / G] = a;
        }
        if (g + 1 < ngrp) {
#pragma unroll
            for (int u = 0; u < CU; ++u)
                xc[u] = xcn[u];
#pragma unroll
            for (int t = 0; t < RW; ++t)
#pragma unroll
                for (int u = 0; u < CU; ++u)
                    x[t][u] = xn[t][u];
        }
    }
    if (rp == 0)
        return;   // uniform over the work-group
    __syncthreads();
    double *rec = A.part + (int64_t)ch.part * rsp * nrhs;
    for (int idx = threadIdx.x; idx < rp * nrhs; idx += blockDim.x) {
        const int l = idx / nrhs, c = idx % nrhs;
        const int g = c / CU, o = (c % CU) * RP + l;
        double s = 0.0;
        for (int w = 0; w < nw; ++w)
            s += wsum[((int64_t)g * nw + w) * NO + o];
        rec[(int64_t)l * nrhs + c] = s;
    }
}

// T of every node of a level with few nodes: one thread per output, summing
// the node's chunk records of that side in chunk order (four partial sums).
// The node solve would otherwise sum a top-level node's many records in one
// work-group.
__global__ __launch_bounds__(LV_THREADS) void level_sum_kernel(LevelArgs A0)
{
    const LevelArgs A = item_args(A0);
    const int64_t loc = blockIdx.x;
    const int64_t h = A.node0 + loc;
    const int r = A.rank[h];
    const int ncnt = A.ncnt, rs = A.rstride;
    const int o = blockIdx.y * LV_THREADS + threadIdx.x;
    if (r == 0 || o >= 2 * r * ncnt)
        return;
    int base, na, nch;
    node_records(A, loc, base, na, nch);
    const int row2 = o / ncnt, c = o % ncnt;
    const int side = row2 < r ? 1 : 0;
    const int l = row2 < r ? row2 : row2 - r;
    const int q1 = side ? base + nch : base + na;
    int q = side ? base + na : base;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (; q + 3 < q1; q += 4) {
        a0 += A.part[((int64_t)q * rs + l) * ncnt + c];
        a1 += A.part[((int64_t)(q + 1) * rs + l) * ncnt + c];
        a2 += A.part[((int64_t)(q + 2) * rs + l) * ncnt + c];
        a3 += A.part[((int64_t)(q + 3) * rs + l) * ncnt + c];
    }
    for (; q < q1; ++q)
        a0 += A.part[((int64_t)q * rs + l) * ncnt + c];
    double *T = A.Tbuf + loc * A.tstride;
    T[(int64_t)(side ? l : rs + l) * ncnt + c] = (a0 + a1) + (a2 + a3);
}

template <int TH>
__global__ __launch_bounds__(TH) void level_solve_kernel(LevelArgs A0)
{
    const LevelArgs A = item_args(A0);
    const int64_t loc = blockIdx.x;
    const int64_t h = A.node0 + loc;
    const int r = A.rank[h];
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    // with gridDim.y > 1 (levels whose T is summed beforehand) every
    // work-group of a node factors M and solves every gridDim.y-th batch of
    // columns; the first one records the factors
    const bool first = blockIdx.y == 0;
    if (r == 0) {
        if (A.factor && tid == 0 && first)
            A.node_ld[h] = 0.0;
        return;
    }
    // LDS sized by the panel's rank: P, Q, N (rs x (rs+1)) and two RHS batches
    extern __shared__ double dyn[];
    const int ldr = A.rstride + 1;
    double *sPb = dyn, *sQb = dyn + A.rstride * ldr, *sNb = dyn + 2 * A.rstride * ldr;
    double *t1b = dyn + 3 * A.rstride * ldr, *t2b = t1b + A.rstride * (LV_CB + 1);
#define sP(i, j) sPb[(i) * ldr + (j)]
#define sQ(i, j) sQb[(i) * ldr + (j)]
#define sN(i, j) sNb[(i) * ldr + (j)]
#define t1(i, c) t1b[(i) * (LV_CB + 1) + (c)]
#define t2(i, c) t2b[(i) * (LV_CB + 1) + (c)]
    __shared__ int piv[RMAX_LDS];
    __shared__ double red[TH / 64];
    __shared__ int sbad;
    const int ncnt = A.ncnt, rs = A.rstride;
    double *T = A.Tbuf + loc * A.tstride;
    // T rows [0, rs): beta side (top); [rs, 2 rs): alpha side (bottom)
    if (!A.tsum) {
        // each output gets a power-of-two group of threads that splits the
        // node's records; groups stay inside one wave for the final sum.
        // The node's records are its alpha chunks, then its beta chunks, so
        // each side is one contiguous range (na = alpha chunks).
        int base, na, nch;
        node_records(A, loc, base, na, nch);
        const int nout = 2 * r * ncnt;
        int G = 1;
        while (G < 64 && G * 2 * nout <= TH && G < nch)
            G *= 2;
        const int per = TH / G;   // outputs per pass
        const int sub = tid % G;
        for (int o0 = 0; o0 < nout; o0 += per) {
            const int o = o0 + tid / G;
            double acc = 0.0;
            int side = 0, l = 0, c = 0;
            if (o < nout) {
                int row2 = o / ncnt;
                c = o % ncnt;
                side = row2 < r ? 1 : 0;
                l = row2 < r ? row2 : row2 - r;
                const int q1 = side ? base + nch : base + na;
                int q = (side ? base + na : base) + sub;
                // four independent partial sums keep several loads in flight
                double a1 = 0.0, a2 = 0.0, a3 = 0.0;
                for (; q + 3 * G < q1; q += 4 * G) {
                    acc += A.part[((int64_t)q * rs + l) * ncnt + c];
                    a1 += A.part[((int64_t)(q + G) * rs + l) * ncnt + c];
                    a2 += A.part[((int64_t)(q + 2 * G) * rs + l) * ncnt + c];
                    a3 += A.part[((int64_t)(q + 3 * G) * rs + l) * ncnt + c];
                }
                for (; q < q1; q += G)
                    acc += A.part[((int64_t)q * rs + l) * ncnt + c];
                acc = (acc + a1) + (a2 + a3);
            }
            for (int off = G / 2; off > 0; off >>= 1)
                acc += __shfl_xor(acc, off, 64);
            if (o < nout && sub == 0)
                T[(int64_t)(side ? l : rs + l) * ncnt + c] = acc;
        }
    }
    __threadfence_block();
    __syncthreads();
    double *sm = A.small + h * A.sstride;   // [N_LU r*r | P r*r | Q r*r | piv r]
    if (A.factor) {
        const int cp = A.nrhs;   // the child panel's columns follow the updated ones
        for (int idx = tid; idx < r * r; idx += TH) {
            int i = idx / r, j = idx % r;
            sP(i, j) = T[(int64_t)i * ncnt + cp + j];
            sQ(i, j) = T[(int64_t)(rs + i) * ncnt + cp + j];
        }
        if (tid == 0)
            sbad = 0;
        __syncthreads();
        for (int idx = tid; idx < r * r; idx += TH) {
            int i = idx / r, j = idx % r;
            double a = (i == j) ? 1.0 : 0.0;
            for (int k = 0; k < r; ++k)
                a -= sQ(i, k) * sP(k, j);
            sN(i, j) = a;
        }
        __syncthreads();
        // LU with partial pivoting (rows swapped in place)
        for (int k = 0; k < r; ++k) {
            if (tid == 0) {
                int p = k;
                double best = fabs(sN(k, k));
                for (int i = k + 1; i < r; ++i)
                    if (fabs(sN(i, k)) > best) {
                        best = fabs(sN(i, k));
                        p = i;
                    }
                piv[k] = p;
                if (best == 0.0)
                    sbad = 1;
            }
            __syncthreads();
            int p = piv[k];
            if (p != k)
                for (int j = tid; j < r; j += TH) {
                    double a = sN(k, j);
                    sN(k, j) = sN(p, j);
                    sN(p, j) = a;
                }
            __syncthreads();
            double pv = sN(k, k);
            for (int i = k + 1 + tid; i < r; i += TH)
                if (pv != 0.0)
                    sN(i, k) /= pv;
            __syncthreads();
            int tr = r - k - 1;
            for (int idx = tid; idx < tr * tr; idx += TH) {
                int i = k + 1 + idx / tr, j = k + 1 + idx % tr;
                sN(i, j) -= sN(i, k) * sN(k, j);
            }
            __syncthreads();
        }
        // log det M = log det(I - QP); it must be positive for an SPD C
        double lg = 0.0;
        int neg = 0;
        for (int i = tid; i < r; i += TH) {
            double u = sN(i, i);
            lg += log(fabs(u));
            neg += (u < 0.0) ? 1 : 0;
            neg += (piv[i] != i) ? 1 : 0;
        }
        lg = wave_sum(lg);
        for (int off = 32; off > 0; off >>= 1)
            neg += __shfl_xor(neg, off, 64);
        if (lane == 0) {
            red[wid] = lg;
            if (neg & 1)
                atomicOr(&sbad, 2);
        }
        __syncthreads();
        if (tid == 0 && first) {
            double v = red[0];
            for (int w = 1; w < TH / 64; ++w)
                v += red[w];
            if (sbad) {
                atomicOr(A.status, DS_NOTSPD_NODE);
                v = __builtin_nan("");
            }
            A.node_ld[h] = v;
        }
        if (first) {
            for (int idx = tid; idx < r * r; idx += TH) {
                int i = idx / r, j = idx % r;
                sm[idx] = sN(i, j);
                sm[r * r + idx] = sP(i, j);
                sm[2 * r * r + idx] = sQ(i, j);
            }
            for (int i = tid; i < r; i += TH)
                sm[3 * r * r + i] = (double)piv[i];
        }
    } else {
        for (int idx = tid; idx < r * r; idx += TH) {
            int i = idx / r, j = idx % r;
            sN(i, j) = sm[idx];
            sP(i, j) = sm[r * r + idx];
            sQ(i, j) = sm[2 * r * r + idx];
        }
        for (int i = tid; i < r; i += TH)
            piv[i] = (int)sm[3 * r * r + i];
    }
    __syncthreads();
    // S = M^{-1} T on the columns to update, in batches
    double *S = A.Sbuf + loc * A.tstride;
    const int nrhs = A.nrhs;
    for (int c0 = blockIdx.y * LV_CB; c0 < nrhs; c0 += gridDim.y * LV_CB) {
        const int nb = min(LV_CB, nrhs - c0);
        for (int idx = tid; idx < r * nb; idx += TH) {
            int i = idx / nb, c = idx % nb;
            t1(i, c) = T[(int64_t)i * ncnt + c0 + c];
        }
        __syncthreads();
        // t2 := t2 - Q t1, with the row permutation of the LU applied after
        for (int idx = tid; idx < r * nb; idx += TH) {
            int i = idx / nb, c = idx % nb;
            double a = T[(int64_t)(rs + i) * ncnt + c0 + c];
            for (int k = 0; k < r; ++k)
                a -= sQ(i, k) * t1(k, c);
            t2(i, c) = a;
        }
        __syncthreads();
        if (tid < nb) {
            int c = tid;
            for (int k = 0; k < r; ++k) {
                int p = piv[k];
                if (p != k) {
                    double a = t2(k, c);
                    t2(k, c) = t2(p, c);
                    t2(p, c) = a;
                }
            }
            for (int i = 1; i < r; ++i) {
                double a = t2(i, c);
                for (int k = 0; k < i; ++k)
                    a -= sN(i, k) * t2(k, c);
                t2(i, c) = a;
            }
            for (int i = r - 1; i >= 0; --i) {
                double a = t2(i, c);
                for (int k = i + 1; k < r; ++k)
                    a -= sN(i, k) * t2(k, c);
                t2(i, c) = a / sN(i, i);
            }
        }
        __syncthreads();
        for (int idx = tid; idx < r * nb; idx += TH) {
            int i = idx / nb, c = idx % nb;
            double a = t1(i, c);
            for (int k = 0; k < r; ++k)
                a -= sP(i, k) * t2(k, c);
            S[(int64_t)i * nrhs + c0 + c] = a;
            S[(int64_t)(rs + i) * nrhs + c0 + c] = t2(i, c);
        }
        __syncthreads();
    }
}
#undef sP
#undef sQ
#undef sN
#undef t1
#undef t2

// a - sum_{k < r} x(k) y(k), the terms subtracted in order of k, with the
// operand loads of 8 terms issued together (the operands of these node-solve
// products come from HBM and L2, and one term at a time would wait on every
// load)
template <typename FX, typename FY>
__device__ __forceinline__ double dot_sub(double a, int r, FX x, FY y)
{
    int k = 0;
    for (; k + 8 <= r; k += 8) {
        double xv[8], yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            xv[u] = x(k + u);
            yv[u] = y(k + u);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            a -= xv[u] * yv[u];
    }
    for (; k < r; ++k)
        a -= x(k) * y(k);
    return a;
}

// Node solves of levels whose rank is above RMAX_LDS (the LDS path's bound).
// The node's matrices live in its slot of the small-factor store (HBM),
//   [N^{-1} (r x r) | P | Q | N, overwritten by its LU | pivots (r)],
// all row-major.  Factoring: P and Q from T, N = I - Q P, LU with partial
// pivoting under the LDS path's rules (first largest pivot, rows swapped in
// place), log det M = log det N (its sign checked as there), and N^{-1} from
// the triangular solves of the permuted identity, one column per thread.
// Every call then forms S = M^{-1} T for the columns to update as
//   u = t2 - Q t1 (into S's top rows), s2 = N^{-1} u, s1 = t1 - P s2,
// so the solves are products.  T is summed beforehand (level_sum_kernel).
// Within the work-group, values written to HBM by one thread are read by
// others only after a barrier (work-group scope acquire/release).
constexpr int LVW_TH = 256;

__global__ __launch_bounds__(LVW_TH) void level_solve_wide_kernel(LevelArgs A0)
{
    const LevelArgs A = item_args(A0);
    const int64_t loc = blockIdx.x;
    const int64_t h = A.node0 + loc;
    const int r = A.rank[h];
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (r == 0) {
        if (A.factor && tid == 0)
            A.node_ld[h] = 0.0;
        return;
    }
    __shared__ int piv[RMAX_ABS];
    __shared__ double sbv[LVW_TH / 64];
    __shared__ int sbi[LVW_TH / 64];
    __shared__ double red[LVW_TH / 64];
    __shared__ int sneg[LVW_TH / 64];
    __shared__ int sbad;
    const int ncnt = A.ncnt, rs = A.rstride, nrhs = A.nrhs;
    const double *T = A.Tbuf + loc * A.tstride;
    double *sm = A.small + h * A.sstride;
    const int64_t rr = (int64_t)r * r;
    double *Ninv = sm, *P = sm + rr, *Q = sm + 2 * rr, *N = sm + 3 * rr;
    if (A.factor) {
        const int cp = nrhs;   // the child panel's columns follow the updated ones
        for (int64_t idx = tid; idx < rr; idx += LVW_TH) {
            const int i = (int)(idx / r), j = (int)(idx % r);
            P[idx] = T[(int64_t)i * ncnt + cp + j];
            Q[idx] = T[(int64_t)(rs + i) * ncnt + cp + j];
        }
        if (tid == 0)
            sbad = 0;
        __syncthreads();
        for (int64_t idx = tid; idx < rr; idx += LVW_TH) {
            const int i = (int)(idx / r), j = (int)(idx % r);
            const double *qi = Q + (int64_t)i * r;
            N[idx] = dot_sub((i == j) ? 1.0 : 0.0, r, [&](int k) { return qi[k]; },
                             [&](int k) { return P[(int64_t)k * r + j]; });
        }
        __syncthreads();
        for (int k = 0; k < r; ++k) {
            // pivot: the first largest |N(i, k)|, i >= k
            double bv = -1.0;
            int bi = r;
            for (int i = k + tid; i < r; i += LVW_TH) {
                const double v = fabs(N[(int64_t)i * r + k]);
                if (v > bv) {
                    bv = v;
                    bi = i;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            if (lane == 0) {
                sbv[wid] = bv;
                sbi[wid] = bi;
            }
            __syncthreads();
            if (tid == 0) {
                double best = sbv[0];
                int p = sbi[0];
                for (int w = 1; w < LVW_TH / 64; ++w)
                    if (sbv[w] > best || (sbv[w] == best && sbi[w] < p)) {
                        best = sbv[w];
                        p = sbi[w];
                    }
                piv[k] = p;
                if (best == 0.0)
                    sbad = 1;
            }
            __syncthreads();
            const int p = piv[k];
            if (p != k)
                for (int j = tid; j < r; j += LVW_TH) {
                    const double a = N[(int64_t)k * r + j];
                    N[(int64_t)k * r + j] = N[(int64_t)p * r + j];
                    N[(int64_t)p * r + j] = a;
                }
            __syncthreads();
            const double pv = N[(int64_t)k * r + k];
            for (int i = k + 1 + tid; i < r; i += LVW_TH)
                if (pv != 0.0)
                    N[(int64_t)i * r + k] /= pv;
            __syncthreads();
            const int tr = r - k - 1;
            for (int64_t idx = tid; idx < (int64_t)tr * tr; idx += LVW_TH) {
                const int i = k + 1 + (int)(idx / tr), j = k + 1 + (int)(idx % tr);
                N[(int64_t)i * r + j] -= N[(int64_t)i * r + k] * N[(int64_t)k * r + j];
            }
            __syncthreads();
        }
        // log det M = log det(I - QP); it must be positive for an SPD C
        double lg = 0.0;
        int neg = 0;
        for (int i = tid; i < r; i += LVW_TH) {
            const double u = N[(int64_t)i * r + i];
            lg += log(fabs(u));
            neg += (u < 0.0) ? 1 : 0;
            neg += (piv[i] != i) ? 1 : 0;
            sm[4 * rr + i] = (double)piv[i];
        }
        lg = wave_sum(lg);
        for (int off = 32; off > 0; off >>= 1)
            neg += __shfl_xor(neg, off, 64);
        if (lane == 0) {
            red[wid] = lg;
            sneg[wid] = neg;
        }
        __syncthreads();
        if (tid == 0) {
            double v = red[0];
            int ng = sneg[0];
            for (int w = 1; w < LVW_TH / 64; ++w) {
                v += red[w];
                ng += sneg[w];
            }
            if (sbad || (ng & 1)) {
                atomicOr(A.status, DS_NOTSPD_NODE);
                v = __builtin_nan("");
            }
            A.node_ld[h] = v;
        }
        // N^{-1}: column c solves N x = e_c (rows permuted as in the LU)
        for (int c = tid; c < r; c += LVW_TH) {
            for (int i = 0; i < r; ++i)
                Ninv[(int64_t)i * r + c] = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < r; ++k) {
                const int p = piv[k];
                if (p != k) {
                    const double a = Ninv[(int64_t)k * r + c];
                    Ninv[(int64_t)k * r + c] = Ninv[(int64_t)p * r + c];
                    Ninv[(int64_t)p * r + c] = a;
                }
            }
            for (int i = 1; i < r; ++i) {
                double a = Ninv[(int64_t)i * r + c];
                for (int k = 0; k < i; ++k)
                    a -= N[(int64_t)i * r + k] * Ninv[(int64_t)k * r + c];
                Ninv[(int64_t)i * r + c] = a;
            }
            for (int i = r - 1; i >= 0; --i) {
                double a = Ninv[(int64_t)i * r + c];
                for (int k = i + 1; k < r; ++k)
                    a -= N[(int64_t)i * r + k] * Ninv[(int64_t)k * r + c];
                Ninv[(int64_t)i * r + c] = a / N[(int64_t)i * r + i];
            }
        }
        __syncthreads();
    }
    // S = M^{-1} T on the columns to update
    double *S = A.Sbuf + loc * A.tstride;
    const int64_t nout = (int64_t)r * nrhs;
    for (int64_t idx = tid; idx < nout; idx += LVW_TH) {   // u = t2 - Q t1
        const int i = (int)(idx / nrhs), c = (int)(idx % nrhs);
        const double *qi = Q + (int64_t)i * r;
        S[(int64_t)i * nrhs + c] =
            dot_sub(T[(int64_t)(rs + i) * ncnt + c], r, [&](int k) { return qi[k]; },
                    [&](int k) { return T[(int64_t)k * ncnt + c]; });
    }
    __syncthreads();
    for (int64_t idx = tid; idx < nout; idx += LVW_TH) {   // s2 = N^{-1} u
        const int i = (int)(idx / nrhs), c = (int)(idx % nrhs);
        const double *ni = Ninv + (int64_t)i * r;
        S[(int64_t)(rs + i) * nrhs + c] =
            dot_sub(0.0, r, [&](int k) { return -ni[k]; },
                    [&](int k) { return S[(int64_t)k * nrhs + c]; });
    }
    __syncthreads();
    for (int64_t idx = tid; idx < nout; idx += LVW_TH) {   // s1 = t1 - P s2
        const int i = (int)(idx / nrhs), c = (int)(idx % nrhs);
        const double *pi = P + (int64_t)i * r;
        S[(int64_t)i * nrhs + c] =
            dot_sub(T[(int64_t)i * ncnt + c], r, [&](int k) { return pi[k]; },
                    [&](int k) { return S[(int64_t)(rs + k) * nrhs + c]; });
    }
}

// Node solves of levels whose rank is above RMAX_LDS and at most LVG_RMAX,
// with N in LDS: the same small-factor store as level_solve_wide_kernel
// ([N^{-1} | P | Q | unused | unused]) and the same products, but N = I - Q P
// is inverted in place by Gauss-Jordan elimination with partial pivoting
// (first largest |N(i, k)| over i >= k, rows swapped), on 1024 threads with
// three barriers per pivot.  Its pivots are those of the LU factorization with
// the same pivoting, so log det M = sum log |pivot| and the sign of det N is
// the parity of the negative pivots and the row swaps, checked as on the
// other paths.  The eliminated array is N^{-1} with permuted columns: column
// c of N^{-1} is its column sig(c), sig(c) = s_{r-1}(... s_0(c)), s_k the
// swap of k and the k-th pivot row.
constexpr int LVG_TH = 1024;
constexpr int LVG_RMAX = 128;

static_assert(LVG_TH % LVG_RMAX == 0 && LVG_RMAX <= LVG_TH, "thread map of the Gauss-Jordan kernel");

static size_t gj_lds(int rs)
{
    return sizeof(double) * ((size_t)rs * (rs + 1) + 3 * (size_t)rs) + sizeof(int) * 2 * (size_t)rs;
}

__global__ __launch_bounds__(LVG_TH) void level_solve_gj_kernel(LevelArgs A0)
{
    const LevelArgs A = item_args(A0);
    const int64_t loc = blockIdx.x;
    const int64_t h = A.node0 + loc;
    const int r = A.rank[h];
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    // element loops: thread (ti, tj) takes column tj of rows ti, ti + 8, ...
    constexpr int TI = LVG_TH / LVG_RMAX;
    const int tj = tid & (LVG_RMAX - 1), ti = tid / LVG_RMAX;
    if (r == 0) {
        if (A.factor && tid == 0)
            A.node_ld[h] = 0.0;
        return;
    }
    extern __shared__ double gsh[];
    const int ld = r + 1;
    double *sA = gsh;                       // r x ld, row-major
    double *rowp = sA + (int64_t)r * ld;    // step k: the pivot row (row p before the swap)
    double *rowo = rowp + r;                // step k: row k before the swap (moves to row p)
    double *colk = rowo + r;                // step k: column k after the swap; then the pivots
    int *piv = (int *)(colk + r);
    int *sig = piv + r;
    __shared__ double s_pv[LVG_RMAX], red[LVG_TH / 64];
    __shared__ int sneg[LVG_TH / 64], s_bad;
    const int ncnt = A.ncnt, rs = A.rstride, nrhs = A.nrhs;
    const double *T = A.Tbuf + loc * A.tstride;
    double *sm = A.small + h * A.sstride;
    const int64_t rr = (int64_t)r * r;
    double *Ninv = sm, *P = sm + rr, *Q = sm + 2 * rr;
    if (A.factor) {
        const int cp = nrhs;   // the child panel's columns follow the updated ones
        // P and Q into the store, Q also into sA; then N = I - Q P with
        // thread (ti, tj) holding rows ti + 8 m of column tj in registers,
        // Q's entries from LDS (one address per wave) and P's rows from T,
        // 8 rows per round
        if (tj < r)
            for (int i = ti; i < r; i += TI) {
                const double q = T[(int64_t)(rs + i) * ncnt + cp + tj];
                P[(int64_t)i * r + tj] = T[(int64_t)i * ncnt + cp + tj];
                Q[(int64_t)i * r + tj] = q;
                sA[i * ld + tj] = q;
            }
        if (tid == 0)
            s_bad = 0;
        __syncthreads();
        constexpr int NM = LVG_RMAX / TI;
        double acc[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m)
            acc[m] = (ti + TI * m == tj) ? 1.0 : 0.0;
        if (tj < r) {
            for (int k0 = 0; k0 < r; k0 += 8) {
                double pv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    pv[u] = (k0 + u < r) ? T[(int64_t)(k0 + u) * ncnt + cp + tj] : 0.0;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (k0 + u < r)
#pragma unroll
                        for (int m = 0; m < NM; ++m) {
                            const int i = ti + TI * m;
                            if (i < r)
                                acc[m] -= sA[i * ld + k0 + u] * pv[u];
                        }
            }
        }
        __syncthreads();   // every read of Q in sA done
        if (tj < r)
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                const int i = ti + TI * m;
                if (i < r)
                    sA[i * ld + tj] = acc[m];
            }
        __syncthreads();
        for (int k = 0; k < r; ++k) {
            if (wid == 0) {   // pivot: the first largest |N(i, k)|, i >= k
                double bv = -1.0;
                int bi = r;
                for (int i = k + lane; i < r; i += 64) {
                    const double v = fabs(sA[i * ld + k]);
                    if (v > bv) {
                        bv = v;
                        bi = i;
                    }
                }
                for (int off = 32; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(bv, off, 64);
                    const int oi = __shfl_xor(bi, off, 64);
                    if (ov > bv || (ov == bv && oi < bi)) {
                        bv = ov;
                        bi = oi;
                    }
                }
                if (lane == 0) {
                    const int p = bi < r ? bi : k;
                    piv[k] = p;
                    const double pv = sA[p * ld + k];
                    if (!(bv > 0.0))
                        s_bad = 1;
                    s_pv[k] = pv != 0.0 ? pv : 1.0;   // flagged above; values stay finite
                }
            }
            __syncthreads();
            // rows k and p swapped: the pivot row, the row it displaces and
            // column k as they are after the swap, read before any write
            const int p = piv[k];
            if (tid < r) {
                rowp[tid] = sA[p * ld + tid];
                rowo[tid] = sA[k * ld + tid];
                const int src = (tid == k) ? p : (tid == p) ? k : tid;
                colk[tid] = sA[src * ld + k];
            }
            __syncthreads();
            // the elimination: every entry is written by the thread that
            // reads it, rows k and p (p != k) from the saved copies
            const double inv = 1.0 / s_pv[k];
            if (tj < r) {
                const double rk = rowp[tj] * inv;
                for (int i = ti; i < r; i += TI) {
                    double v;
                    if (i == k) {
                        v = (tj == k) ? inv : rk;
                    } else {
                        const double old = (i == p) ? rowo[tj] : sA[i * ld + tj];
                        v = (tj == k) ? -colk[i] * inv : old - colk[i] * rk;
                    }
                    sA[i * ld + tj] = v;
                }
            }
            __syncthreads();
        }
        // column permutation of the inverse, log det and its sign
        double lg = 0.0;
        int neg = 0;
        if (tid < r) {
            int v = tid;
            for (int k = 0; k < r; ++k) {
                const int pk = piv[k];
                v = (v == k) ? pk : (v == pk) ? k : v;
            }
            sig[tid] = v;
            lg = log(fabs(s_pv[tid]));
            neg = (s_pv[tid] < 0.0 ? 1 : 0) + (piv[tid] != tid ? 1 : 0);
        }
        lg = wave_sum(lg);
        for (int off = 32; off > 0; off >>= 1)
            neg += __shfl_xor(neg, off, 64);
        if (lane == 0) {
            red[wid] = lg;
            sneg[wid] = neg;
        }
        __syncthreads();
        if (tid == 0) {
            double v = 0.0;
            int ng = 0;
            for (int w = 0; w < LVG_TH / 64; ++w) {
                v += red[w];
                ng += sneg[w];
            }
            if (s_bad || (ng & 1)) {
                atomicOr(A.status, DS_NOTSPD_NODE);
                v = __builtin_nan("");
            }
            A.node_ld[h] = v;
        }
        if (tj < r)
            for (int i = ti; i < r; i += TI)
                Ninv[(int64_t)i * r + tj] = sA[i * ld + sig[tj]];
    }
    // S = M^{-1} T on the columns to update (N^{-1} from LDS when just
    // factored, else from the store)
    double *S = A.Sbuf + loc * A.tstride;
    const int64_t nout = (int64_t)r * nrhs;
    for (int64_t idx = tid; idx < nout; idx += LVG_TH) {   // u = t2 - Q t1
        const int i = (int)(idx / nrhs), c = (int)(idx % nrhs);
        const double *qi = Q + (int64_t)i * r;
        S[(int64_t)i * nrhs + c] =
            dot_sub(T[(int64_t)(rs + i) * ncnt + c], r, [&](int k) { return qi[k]; },
                    [&](int k) { return T[(int64_t)k * ncnt + c]; });
    }
    __syncthreads();
    for (int64_t idx = tid; idx < nout; idx += LVG_TH) {   // s2 = N^{-1} u
        const int i = (int)(idx / nrhs), c = (int)(idx % nrhs);
        double a;
        if (A.factor) {
            const double *ni = sA + i * ld;
            a = dot_sub(0.0, r, [&](int k) { return -ni[sig[k]]; },
                        [&](int k) { return S[(int64_t)k * nrhs + c]; });
        } else {
            const double *ni = Ninv + (int64_t)i * r;
            a = dot_sub(0.0, r, [&](int k) { return -ni[k]; },
                        [&](int k) { return S[(int64_t)k * nrhs + c]; });
        }
        S[(int64_t)(rs + i) * nrhs + c] = a;
    }
    __syncthreads();
    for (int64_t idx = tid; idx < nout; idx += LVG_TH) {   // s1 = t1 - P s2
        const int i = (int)(idx / nrhs), c = (int)(idx % nrhs);
        const double *pi = P + (int64_t)i * r;
        S[(int64_t)i * nrhs + c] =
            dot_sub(T[(int64_t)i * ncnt + c], r, [&](int k) { return pi[k]; },
                    [&](int k) { return S[(int64_t)(rs + k) * nrhs + c]; });
    }
}

// Wide ranks (panel rank above 8, e.g. 2-D kernels or tight tolerances) on
// FP64 MFMA (v_mfma_f64_16x16x4; lane l = 16 q + r supplies A[r][q] and
// B[q][r] of a 16 x 4 by 4 x 16 step and holds D[q + 4 t][r], t < 4).
typedef double lv_d4 __attribute__((ext_vector_type(4)));
constexpr int LVM_UNT = 8;  // 16-column tiles per work-group in the update

// T_part[chunk] = W_chunk^T X_chunk with both operands staged in LDS: the
// chunk's rows go through 64 at a time, lane = row, so every load of a
// column-major panel is 512 contiguous bytes; wave w stages columns w, w + 4,
// ... of this work-group's 64 CPW columns and ranks w, w + 4, ... of its rank
// group (16 MT ranks).  The next step's loads are issued into registers
// before the current step's MFMAs (16 steps of 4 rows from LDS), so they are
// in flight while the matrix cores work.  Wave w owns column tiles w, w + 4;
// blockIdx.y = column block + (column blocks) x rank group.  The records are
// those of the other reductions.
constexpr int RL_ROWS = 64;

template <typename PT, int MT, int CPW>
__global__ __launch_bounds__(LV_THREADS) void level_reduce_lds_kernel(LevelArgs A0)
{
    constexpr int NCOL = 64 * CPW;   // columns per work-group
    constexpr int NR = 16 * MT;      // ranks per group
    constexpr int XPT = NCOL / 4, WPT = NR / 4;   // values each lane stages per step
    const LevelArgs A = item_args(A0);
    const Chunk ch = A.chunks[blockIdx.x];
    const int r = A.rank[ch.node];
    const int ncb = (A.ncnt + NCOL - 1) / NCOL;
    const int r0 = NR * (int)(blockIdx.y / ncb);
    const int c0 = NCOL * (int)(blockIdx.y % ncb);
    if (r == 0 || r0 >= r)
        return;   // the whole work-group
    __shared__ double sX[RL_ROWS][NCOL + 1];
    __shared__ double sW[RL_ROWS][NR + 1];
    __shared__ int scol[NCOL];
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lq = lane >> 4;
    const int64_t n = A.n;
    const PT *__restrict__ Xp = (const PT *)A.Xt;
    const double *__restrict__ Wp = A.W + A.colW * n;
    // columns past the last one read the first column and store zero
    for (int c = tid; c < NCOL; c += LV_THREADS)
        scol[c] = A.cols[c0 + c < A.ncnt ? c0 + c : 0];
    __syncthreads();
    double xr[XPT], wr[WPT];
    auto load = [&](int64_t i0) {
        const int64_t i = i0 + lane;
        const bool ok = i < ch.hi;
        const int64_t is = ok ? i : ch.lo;
#pragma unroll
        for (int k = 0; k < XPT; ++k) {
            const int c = wid + 4 * k;
            const double v = (double)Xp[(int64_t)scol[c] * n + is];
            xr[k] = (ok && c0 + c < A.ncnt) ? v : 0.0;
        }
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int l = r0 + wid + 4 * k;
            const double v = Wp[(int64_t)(l < r ? l : 0) * n + is];
            wr[k] = (ok && l < r) ? v : 0.0;
        }
    };
    lv_d4 acc[CPW][MT];
#pragma unroll
    for (int j = 0; j < CPW; ++j)
#pragma unroll
        for (int m = 0; m < MT; ++m)
            acc[j][m] = lv_d4{0.0, 0.0, 0.0, 0.0};
    load(ch.lo);
    for (int64_t i0 = ch.lo; i0 < ch.hi; i0 += RL_ROWS) {
        __syncthreads();   // the previous step's operands consumed
#pragma unroll
        for (int k = 0; k < XPT; ++k)
            sX[lane][wid + 4 * k] = xr[k];
#pragma unroll
        for (int k = 0; k < WPT; ++k)
            sW[lane][wid + 4 * k] = wr[k];
        __syncthreads();
        if (i0 + RL_ROWS < ch.hi)
            load(i0 + RL_ROWS);
#pragma unroll 4
        for (int ks = 0; ks < RL_ROWS / 4; ++ks) {
            const int kr = 4 * ks + lq;
            double a[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m)
                a[m] = sW[kr][16 * m + lr];
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const double b = sX[kr][16 * (wid + 4 * j) + lr];
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    acc[j][m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b, acc[j][m], 0, 0, 0);
            }
        }
    }
    // lane (lr, lq) holds T[rank r0 + 16 m + lq + 4 t][column c0 + 16 (wid + 4 j) + lr]
    double *rec = A.part + (int64_t)ch.part * A.rstride * A.ncnt;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int c = c0 + 16 * (wid + 4 * j) + lr;
        if (c < A.ncnt) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int l = r0 + 16 * m + lq + 4 * t;
                    if (l < r)
                        rec[(int64_t)l * A.ncnt + c] = acc[j][m][t];
                }
        }
    }
}

// X_chunk[:, cols] -= W~_chunk S, as (W~ S)^T = S^T W~^T: M = 16 columns, N =
// 16 rows per tile, K = ranks (4 per step, 4 MT steps: the level's reserved
// rank rounded up).  A work-group takes one chunk and 128 columns: S's slice
// for them in LDS, each wave every fourth row tile, whose W~ operands serve
// the 8 column tiles.
template <typename PT, int MT>
__global__ __launch_bounds__(LV_THREADS) void level_update_mfma_kernel(LevelArgs A0)
{
    const LevelArgs A = item_args(A0);
    PT *__restrict__ Xp = (PT *)A.Xt;
    const Chunk ch = A.chunks[blockIdx.x];
    const int r = A.rank[ch.node];
    const int nrhs = A.nrhs;
    const int cbase = blockIdx.y * LVM_UNT * 16;
    if (r == 0 || cbase >= nrhs)
        return;   // the whole work-group
    constexpr int KS = 4 * MT;   // 4-rank steps per rank chunk
    __shared__ double sS[4 * KS][LVM_UNT * 16 + 1];
    __shared__ int scol[LVM_UNT * 16];
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lq = lane >> 4;
    const int64_t n = A.n;
    const int64_t loc = ch.node - A.node0;
    const double *S = A.Sbuf + loc * A.tstride;
    const int rowoff = ch.side ? A.rstride : 0;   // alpha uses S_top, beta S_bottom
    for (int cc = tid; cc < LVM_UNT * 16; cc += LV_THREADS)
        scol[cc] = cbase + cc < nrhs ? A.cols[cbase + cc] : -1;
    // ranks in chunks of 4 KS (one chunk unless the rank is above 16 MT):
    // S's slice of the chunk in LDS, X updated once per chunk
    for (int r0 = 0; r0 < r; r0 += 4 * KS) {
    if (r0)
        __syncthreads();   // every wave is done with the previous slice
    for (int idx = tid; idx < 4 * KS * LVM_UNT * 16; idx += LV_THREADS) {
        const int l = idx / (LVM_UNT * 16), cc = idx % (LVM_UNT * 16);
        const int col = cbase + cc;
        sS[l][cc] = (r0 + l < r && col < nrhs) ? S[(int64_t)(rowoff + r0 + l) * nrhs + col] : 0.0;
    }
    __syncthreads();
    const int64_t nrt = (ch.hi - ch.lo + 15) >> 4;
    for (int64_t rt = wid; rt < nrt; rt += LV_THREADS / 64) {
        const int64_t i0 = ch.lo + 16 * rt;
        double a[KS];
        const int64_t ia = i0 + lr;
        const bool rok = ia < ch.hi;
        const int64_t is = rok ? ia : ch.lo;
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int l = r0 + 4 * st + lq;
            const double wv = (double)Xp[(A.colW + (l < r ? l : 0)) * n + is];
            a[st] = (l < r && rok) ? wv : 0.0;
        }
#pragma unroll
        for (int j = 0; j < LVM_UNT; ++j) {
            if (cbase + 16 * j >= nrhs)
                break;
            // the transposed product (W~ S)^T = S^T W~^T, so that a lane's
            // results lie along rows: lane (lr, lq) holds row i0 + lr of
            // columns cbase + 16 j + lq + 4 t, and each load or store of X
            // covers 16 consecutive rows of 4 columns
            // the tile's X values loaded first and without a condition (a
            // column past the list reads column 0, a row past the chunk its
            // first row; neither is stored), so the four loads are in flight
            // during the products instead of each waiting in a branch
            int cl[4];
            double xv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                cl[t] = scol[16 * j + lq + 4 * t];
                xv[t] = (double)Xp[(int64_t)(cl[t] >= 0 ? cl[t] : 0) * n + is];
            }
            lv_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int st = 0; st < KS; ++st)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sS[4 * st + lq][16 * j + lr], a[st], acc,
                                                           0, 0, 0);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (rok && cl[t] >= 0)
                    Xp[(int64_t)cl[t] * n + ia] = (PT)(xv[t] - acc[t]);
        }
    }
    }
}

static size_t solve_lds(int rs)
{
    static bool attr = false;   // allow the rank-64 size (about 134 KB) once per process
    if (!attr) {
        HIP_TRY(hipFuncSetAttribute((const void *)level_solve_kernel<LV_SOLVE_TH>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
        HIP_TRY(hipFuncSetAttribute((const void *)level_solve_kernel<64>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
        HIP_TRY(hipFuncSetAttribute((const void *)level_solve_gj_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)gj_lds(LVG_RMAX)));
        attr = true;
    }
    return sizeof(double) * ((size_t)3 * rs * (rs + 1) + (size_t)2 * rs * (LV_CB + 1) + 1);
}

// node solves of one level: levels with many small-rank nodes (few records
// each) on one wave per node, the others on LV_SOLVE_TH threads (whose record
// sums need the loads in flight)
static void launch_solve(Pipeline &P, const LevelArgs &A, unsigned nodes, unsigned ysplit = 1)
{
    if (nodes >= 512 && A.rstride <= 8)
        level_solve_kernel<64><<<dim3(nodes, 1, P.nitems), 64, solve_lds(A.rstride), P.stream>>>(A);
    else
        level_solve_kernel<LV_SOLVE_TH><<<dim3(nodes, ysplit, P.nitems), LV_SOLVE_TH, solve_lds(A.rstride),
                                          P.stream>>>(A);
}

// set once, outside any stream capture
void prime_level_attributes() { (void)solve_lds(1); }

static LevelArgs level_args(Pipeline &P, int d)
{
    const Plan &p = *P.plan;
    LevelArgs A;
    A.n = p.n;
    A.W = wsp<double>(P, P.lay.W);
    A.Xt = P.ws + P.lay.Xt;
    A.cols = wsp<int>(P, P.lay.cols);
    A.colW = p.cofa[d + 1];
    A.rstride = P.rmax[d + 1];
    A.rank = wsp<int>(P, P.lay.rank);
    A.chunks = p.d_lvl[d];
    A.nch = p.d_lvl_nch[d];
    A.base = p.d_lvl_base[d];
    A.node0 = p.first_at(d);
    A.part = wsp<double>(P, P.lay.lvl_part);
    A.Tbuf = wsp<double>(P, P.lay.Tbuf);
    A.Sbuf = wsp<double>(P, P.lay.Sbuf);
    A.small = wsp<double>(P, P.lay.small);
    A.sstride = P.lay.small_stride;
    A.node_ld = wsp<double>(P, P.lay.node_ld);
    A.status = wsp<int>(P, P.lay.status);
    A.B = P.batch;
    A.cgrp = p.red_grp;
    A.rows = p.lvl_rows;
    A.tsum = 0;
    A.cbase = A.cnch = nullptr;
    A.colWp = 0;
    A.rstride_p = 0;
    return A;
}

template <typename PT, int R>
static void reduce_small_rows(int sr, int cu, dim3 grid, hipStream_t s, const LevelArgs &A)
{
    if (sr == 4 && cu == 4)
        level_reduce_small_kernel<PT, R, 4, 4><<<grid, 64, 0, s>>>(A);
    else if (sr == 4)
        level_reduce_small_kernel<PT, R, 4, 8><<<grid, 64, 0, s>>>(A);
    else if (sr == 8 && cu == 4)
        level_reduce_small_kernel<PT, R, 8, 4><<<grid, 64, 0, s>>>(A);
    else if (sr == 8)
        level_reduce_small_kernel<PT, R, 8, 8><<<grid, 64, 0, s>>>(A);
    else if (cu == 4)
        level_reduce_small_kernel<PT, R, 16, 4><<<grid, 64, 0, s>>>(A);
    else
        level_reduce_small_kernel<PT, R, 16, 8><<<grid, 64, 0, s>>>(A);
}

template <typename PT>
static void reduce_small_launch(int R, int sr, int cu, dim3 grid, hipStream_t s, const LevelArgs &A)
{
    if (R == 2)
        reduce_small_rows<PT, 2>(sr, cu, grid, s, A);
    else if (R == 4)
        reduce_small_rows<PT, 4>(sr, cu, grid, s, A);
    else
        reduce_small_rows<PT, 8>(sr, cu, grid, s, A);
}

// the LDS-staged reduction: rank groups of 16 MT (MT = ranks / 16 rounded up,
// at most 4), 64 or 128 columns per work-group
template <typename PT>
static void reduce_lds_launch(unsigned nchunks, unsigned nitems, hipStream_t s, const LevelArgs &A)
{
    const int mt = std::min(4, (A.rstride + 15) / 16);
    const int ngrp = (A.rstride + 16 * mt - 1) / (16 * mt);
    const int cpw = A.ncnt > 64 && mt == 1 ? 2 : 1;   // LDS: at most 75 KB, two groups per CU
    const unsigned ncb = (unsigned)((A.ncnt + 64 * cpw - 1) / (64 * cpw));
    const dim3 grid(nchunks, ncb * ngrp, nitems);
#define RL_LAUNCH(MT, CPW) level_reduce_lds_kernel<PT, MT, CPW><<<grid, LV_THREADS, 0, s>>>(A)
    if (cpw == 1) {
        if (mt == 1) RL_LAUNCH(1, 1);
        else if (mt == 2) RL_LAUNCH(2, 1);
        else if (mt == 3) RL_LAUNCH(3, 1);
        else RL_LAUNCH(4, 1);
    } else {
        RL_LAUNCH(1, 2);
    }
#undef RL_LAUNCH
}

template <typename PT>
static void update_mfma_launch(int mt, dim3 grid, hipStream_t s, const LevelArgs &A)
{
    if (mt == 1)
        level_update_mfma_kernel<PT, 1><<<grid, LV_THREADS, 0, s>>>(A);
    else if (mt == 2)
        level_update_mfma_kernel<PT, 2><<<grid, LV_THREADS, 0, s>>>(A);
    else if (mt == 3)
        level_update_mfma_kernel<PT, 3><<<grid, LV_THREADS, 0, s>>>(A);
    else
        level_update_mfma_kernel<PT, 4><<<grid, LV_THREADS, 0, s>>>(A);
}

template <typename PT, int R, int RP, bool UPD>
static void fused_rows(int rw, dim3 grid, int th, size_t lds, hipStream_t s, const LevelArgs &A)
{
    if (rw == 1)
        level_fused_kernel<PT, R, RP, 1, UPD><<<grid, th, lds, s>>>(A);
    else
        level_fused_kernel<PT, R, RP, 2, UPD><<<grid, th, lds, s>>>(A);
}

// LDS of the fused pass: S (R x nrhs), the waves' sums of every column
// group (LVF_CU columns, RP rows each) and the column list
static size_t fused_lds(int nrhs, int R, int RP)
{
    const size_t groups = (size_t)(nrhs + LVF_CU - 1) / LVF_CU;
    return sizeof(double) * ((size_t)R * nrhs + groups * LVF_MAXW * LVF_CU * RP) +
           sizeof(int) * (size_t)nrhs;
}

// the fused update + parent records: ranks classed as 4 (1..4) or 8 (5..8);
// one row per lane for 256-row chunks, else two, and as many waves as the
// level's longest chunk needs
template <typename PT>
static void fused_launch(Pipeline &P, int d, unsigned nchunks, const LevelArgs &A)
{
    const int R = A.rstride <= 4 ? 4 : 8, RP = A.rstride_p <= 4 ? 4 : 8;
    const int rw = P.plan->lvl_rows <= 256 ? 1 : 2;
    const size_t lds = fused_lds(A.nrhs, R, RP);
    const dim3 grid(nchunks, 1, P.nitems);
    const int nw = std::min(LVF_MAXW, (P.plan->lvl_maxlen[d] + 64 * rw - 1) / (64 * rw));
    const int th = 64 * std::max(nw, 1);
    if (R == 4 && RP == 4)
        fused_rows<PT, 4, 4, true>(rw, grid, th, lds, P.stream, A);
    else if (R == 4)
        fused_rows<PT, 4, 8, true>(rw, grid, th, lds, P.stream, A);
    else if (RP == 4)
        fused_rows<PT, 8, 4, true>(rw, grid, th, lds, P.stream, A);
    else
        fused_rows<PT, 8, 8, true>(rw, grid, th, lds, P.stream, A);
}

// the same pass as a plain reduction (the level's own records, A.ncnt columns)
template <typename PT>
static void fused_reduce_launch(Pipeline &P, int d, unsigned nchunks, const LevelArgs &A)
{
    const int rw = P.plan->lvl_rows <= 256 ? 1 : 2;
    const dim3 grid(nchunks, 1, P.nitems);
    const int nw = std::min(LVF_MAXW, (P.plan->lvl_maxlen[d] + 64 * rw - 1) / (64 * rw));
    const int th = 64 * std::max(nw, 1);
    if (A.rstride <= 4)
        fused_rows<PT, 4, 4, false>(rw, grid, th, fused_lds(A.ncnt, 0, 4), P.stream, A);
    else
        fused_rows<PT, 4, 8, false>(rw, grid, th, fused_lds(A.ncnt, 0, 8), P.stream, A);
}

// whether level d's update also writes level d-1's reduction records: both
// levels of the small-rank kind with S in LDS
static bool fuse_levels(const Pipeline &P, int d)
{
    const Plan &p = *P.plan;
    if (d < 1 || p.lvl[d].empty() || P.cnt[d] <= 0)
        return false;
    const int r = P.rmax[d + 1], rp = P.rmax[d];
    return r > 0 && r <= 8 && rp > 0 && rp <= 8 && fused_lds(P.cnt[d], 8, 8) <= 64 * 1024;
}

// levels of rank above RMAX_LDS: the MFMA reduction over rank groups of 64,
// the record sums, the node solves (N in LDS up to rank LVG_RMAX, else in
// HBM), and the MFMA update over rank chunks of 64
template <typename PT>
static void level_launch_wide(Pipeline &P, int d, LevelArgs A)
{
    const Plan &p = *P.plan;
    const unsigned nchunks = (unsigned)p.lvl[d].size();
    const unsigned nodes = (unsigned)(p.first_at(d + 1) - p.first_at(d));
    if (nchunks) {
        ProfScope ps(P.stream, PS_LVL_REDUCE);
        reduce_lds_launch<PT>(nchunks, P.nitems, P.stream, A);
    }
    {
        ProfScope ps(P.stream, PS_LVL_SOLVE);
        A.tsum = 1;
        if (nchunks) {
            const int most = 2 * A.rstride * A.ncnt;
            level_sum_kernel<<<dim3(nodes, (most + LV_THREADS - 1) / LV_THREADS, P.nitems), LV_THREADS,
                               0, P.stream>>>(A);
        }
        if (A.rstride <= LVG_RMAX) {
            (void)solve_lds(1);   // the dynamic LDS limits, once per process
            level_solve_gj_kernel<<<dim3(nodes, 1, P.nitems), LVG_TH, gj_lds(A.rstride), P.stream>>>(A);
        } else {
            level_solve_wide_kernel<<<dim3(nodes, 1, P.nitems), LVW_TH, 0, P.stream>>>(A);
        }
    }
    if (nchunks && A.nrhs > 0) {
        ProfScope ps(P.stream, PS_LVL_UPDATE);
        level_update_mfma_kernel<PT, 4>
            <<<dim3(nchunks, (A.nrhs + 16 * LVM_UNT - 1) / (16 * LVM_UNT), P.nitems), LV_THREADS, 0,
               P.stream>>>(A);
    }
    HIP_TRY(hipGetLastError());
}

template <typename PT>
static void level_launch_t(Pipeline &P, int d, LevelArgs A, bool fuse_up)
{
    if (A.rstride > RMAX_LDS) {
        level_launch_wide<PT>(P, d, A);
        return;
    }
    const Plan &p = *P.plan;
    const unsigned nchunks = (unsigned)p.lvl[d].size();
    const unsigned nodes = (unsigned)(p.first_at(d + 1) - p.first_at(d));
    const int R = A.rstride <= 2 ? 2 : A.rstride <= 4 ? 4 : A.rstride <= 8 ? 8 : 0;
    const size_t sbytes = sizeof(double) * (size_t)R * A.nrhs;
    const bool small_upd = R > 0 && sbytes <= 48 * 1024;
    if (nchunks && !A.cbase) {
        ProfScope ps(P.stream, PS_LVL_REDUCE);
        const dim3 grid(nchunks, (A.ncnt + p.red_grp - 1) / p.red_grp, P.nitems);
        if (R > 0 && A.factor && fused_lds(A.ncnt, 0, 8) <= 64 * 1024)
            fused_reduce_launch<PT>(P, d, nchunks, A);
        else if (R > 0)
            reduce_small_launch<PT>(R, p.lvl_rows / 64, p.red_cols, grid, P.stream, A);
        else
            reduce_lds_launch<PT>(nchunks, P.nitems, P.stream, A);
    }
    {
        ProfScope ps(P.stream, PS_LVL_SOLVE);
        const double per_node = (double)nchunks / nodes * 2.0 * A.rstride * A.ncnt;
        unsigned ysplit = 1;
        const bool wide = nodes <= LV_SPLIT_NODES && A.nrhs > LV_SPLIT_COLS;
        if (nchunks && (per_node > LV_SUM_MIN || wide)) {
            A.tsum = 1;
            const int most = 2 * A.rstride * A.ncnt;
            level_sum_kernel<<<dim3(nodes, (most + LV_THREADS - 1) / LV_THREADS, P.nitems), LV_THREADS,
                               0, P.stream>>>(A);
            // few nodes with many columns: the column batches go to several
            // work-groups per node, each factoring the node's small matrix
            if (nodes <= LV_SPLIT_NODES && A.nrhs > LV_CB) {
                const unsigned batches = (unsigned)((A.nrhs + LV_CB - 1) / LV_CB);
                ysplit = std::min({batches, LV_SPLIT_GROUPS, std::max(1u, LV_SPLIT_TOTAL / nodes)});
            }
        }
        launch_solve(P, A, nodes, ysplit);
    }
    if (nchunks && A.nrhs > 0) {
        ProfScope ps(P.stream, PS_LVL_UPDATE);
        if (fuse_up)
            fused_launch<PT>(P, d, nchunks, A);
        else if (small_upd && R == 2)
            level_update_small_kernel<PT, 2><<<dim3(nchunks, 1, P.nitems), LV_THREADS, sbytes, P.stream>>>(A, 0);
        else if (small_upd && R == 4)
            level_update_small_kernel<PT, 4><<<dim3(nchunks, 1, P.nitems), LV_THREADS, sbytes, P.stream>>>(A, 0);
        else if (small_upd && R == 8)
            level_update_small_kernel<PT, 8><<<dim3(nchunks, 1, P.nitems), LV_THREADS, sbytes, P.stream>>>(A, 0);
        else
            update_mfma_launch<PT>((A.rstride + 15) / 16,
                                   dim3(nchunks, (A.nrhs + 16 * LVM_UNT - 1) / (16 * LVM_UNT), P.nitems),
                                   P.stream, A);
    }
    HIP_TRY(hipGetLastError());
}

static void level_launch(Pipeline &P, int d, LevelArgs A, bool fuse_up = false)
{
    if (P.plan->f32())
        level_launch_t<float>(P, d, A, fuse_up);
    else
        level_launch_t<double>(P, d, A, fuse_up);
}

void run_levels_factor(Pipeline &P)
{
    P.proj_run = proj_fits(P);
    if (P.proj_run) {
        run_levels_projected(P);
        return;
    }
    const Plan &p = *P.plan;
    bool below = false;   // level d+1's update wrote this level's records
    for (int d = p.L - 1; d >= 0; --d) {
        LevelArgs A = level_args(P, d);
        A.factor = 1;
        A.ncnt = P.cnt[d + 1];
        A.nrhs = P.cnt[d];
        A.tstride = 2 * (int64_t)A.rstride * A.ncnt;
        if (A.rstride == 0) {
            // every block of this level has rank 0: coupling determinants are 1
            const unsigned nodes = (unsigned)(p.first_at(d + 1) - p.first_at(d));
            ProfScope ps(P.stream, PS_LVL_SOLVE);
            launch_solve(P, A, nodes);
            HIP_TRY(hipGetLastError());
            below = false;
            continue;
        }
        if (below) {
            A.cbase = p.d_lvl_base[d + 1];
            A.cnch = p.d_lvl_nch[d + 1];
        }
        const bool fuse = fuse_levels(P, d);
        if (fuse) {
            A.colWp = p.cofa[d];
            A.rstride_p = P.rmax[d];
        }
        level_launch(P, d, A, fuse);
        below = fuse;
    }
}

void run_levels_apply(Pipeline &P)
{
    const Plan &p = *P.plan;
    for (int d = p.L - 1; d >= 0; --d) {
        LevelArgs A = level_args(P, d);
        if (A.rstride == 0)
            continue;
        A.factor = 0;
        A.ncnt = 1;
        A.nrhs = 1;
        A.tstride = 2 * (int64_t)A.rstride;
        level_launch(P, d, A);
    }
}

}  // namespace hodlr
