// Leaf stage: the dense diagonal blocks C_lambda = K(lambda, lambda) +
// sigma^2 I of the finest level (the factor K_kappa of §3.2), their Cholesky
// factors and log-dets, and C_lambda^{-1} applied to the leaf's rows of every
// off-diagonal basis above it and of the right-hand side (§3.3 notes that this
// application, not the small inverse itself, is what costs most at the leaves).
//
// One work-group per leaf.  The block is evaluated on the fly from the
// ordered coordinates straight into LDS as 16 x 16 tiles of its lower
// triangle, factored there on FP64 MFMA, and the basis columns are solved in
// registers, 16 columns per wave at a time.
#include <utility>

#include "common.h"

namespace hodlr {

constexpr int LEAF_SOLVE_T = 64;   // one wave per leaf in the solve with stored factors

struct LeafArgs {
    const double *x;
    int64_t n;
    KParams kp;
    const int64_t *start, *end;
    int64_t leaf0;          // heap index of the first leaf
    const double *W;        // original bases (source columns)
    void *Xt;               // destination columns (float in the mixed form)
    const double *y;        // right-hand side for column 0 (nullable)
    const int *cols;
    int ncols, cbeg;
    double *G;              // packed Cholesky factors (nullable)
    int64_t gstride;
    double *leaf_ld;
    int *status;
    double *L21;            // leaves above LEAF_LDS_MAX: their off-diagonal factor tiles
    BatchArgs B;
};

__device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }

__device__ __forceinline__ int tri_row(int idx)
{
    int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while (tri(i + 1) <= idx)
        ++i;
    while (tri(i) > idx)
        --i;
    return i;
}

// ---------------------------------------------------------------------------
// Blocked FP64 factorization on the matrix cores.  The leaf (padded to a
// multiple of 16 with an identity block) is held in LDS as 16 x 16 tiles;
// every tile product is four v_mfma_f64_16x16x4 instructions.
//
// MFMA operand layout (lane l, r = l % 16, q = l / 16, kb = 0..3, k = q + 4 kb):
//   A operand A[r][k], B operand B[k][r]; result element t is D[q + 4 t][r].
// Storage: factor tiles column-major, right-hand-side tiles row-major, both
// with leading dimension TLD (17 doubles: conflict-free column accesses).
// With that storage, "A = tile" and "B = tile^T" (factor tiles) or "B = tile"
// (right-hand-side tiles) all read  ptr[k * TLD + r].
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int TLD = 17;
constexpr int TSZ = 16 * TLD;
constexpr int NT_MAX = LEAF_LDS_MAX / 16;           // 8 row tiles
constexpr int NTRI = NT_MAX * (NT_MAX + 1) / 2;     // 36 lower tiles
constexpr int LEAF_MT = 256;                        // threads of the factor kernel
constexpr int LEAF_MW = LEAF_MT / 64;               // its waves

__device__ __forceinline__ int tix(int I, int K) { return I * (I + 1) / 2 + K; }

// acc += op(A) * B^T, op(A) = A or A^T, tiles column-major with leading
// dimension LD (TLD in LDS, 16 for the tiles a large leaf keeps in HBM)
template <bool TA, int LDA = TLD, int LDB = TLD>
__device__ __forceinline__ d4 tile_mma(const double *A, const double *B, d4 acc)
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const int k = q + 4 * kb;
        double a = TA ? A[r * LDA + k] : A[k * LDA + r];
        double b = B[k * LDB + r];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// The FP64 MFMA's last operand carries negate modifiers for A, B and C (bits
// 0-2) on this target; NEG_A gives acc - A B in one instruction.
constexpr int MFMA_NEG_A = 1;

// T1 -= A1 B1^T and (TWO) T2 -= A2 B2^T, tiles in LDS (column-major, leading
// dimension TLD): every LDS read of both products is issued before the first
// MFMA, the products run interleaved from the tiles' own values (negated A
// operand), and T1, T2 are written back.
template <bool TWO>
__device__ __forceinline__ void tile_sub2(double *T1, const double *A1, const double *B1, double *T2,
                                          const double *A2, const double *B2)
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    d4 c1, c2 = {0.0, 0.0, 0.0, 0.0};
    double a1[4], b1[4], a2[4], b2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        c1[t] = T1[r * TLD + q + 4 * t];
        if (TWO)
            c2[t] = T2[r * TLD + q + 4 * t];
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const int k = q + 4 * kb;
        a1[kb] = A1[k * TLD + r];
        b1[kb] = B1[k * TLD + r];
        if (TWO) {
            a2[kb] = A2[k * TLD + r];
            b2[kb] = B2[k * TLD + r];
        }
    }
    // last argument 1: the instruction negates its A operand
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[kb], b1[kb], c1, 0, 0, MFMA_NEG_A);
        if (TWO)
            c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[kb], b2[kb], c2, 0, 0, MFMA_NEG_A);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        T1[r * TLD + q + 4 * t] = c1[t];
        if (TWO)
            T2[r * TLD + q + 4 * t] = c2[t];
    }
}

// T1 = T1 D^T and (TWO) T2 = T2 D^T with one D (the panel of a block column)
template <bool TWO>
__device__ __forceinline__ void tile_panel2(double *T1, double *T2, const double *D)
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    d4 c1 = {0.0, 0.0, 0.0, 0.0}, c2 = {0.0, 0.0, 0.0, 0.0};
    double a1[4], a2[4], b[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const int k = q + 4 * kb;
        a1[kb] = T1[k * TLD + r];
        if (TWO)
            a2[kb] = T2[k * TLD + r];
        b[kb] = D[k * TLD + r];
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[kb], b[kb], c1, 0, 0, 0);
        if (TWO)
            c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[kb], b[kb], c2, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        T1[r * TLD + q + 4 * t] = c1[t];
        if (TWO)
            T2[r * TLD + q + 4 * t] = c2[t];
    }
}

// (I, K) of trailing task `task` at step J: tiles J < K <= I in packed order,
// the look-ahead tile (J+1, J+1) skipped
__device__ __forceinline__ void trail_tile(int task, int J, int &I, int &K)
{
    const int tt = task + 1;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= tt)
        ++i;
    K = tt - i * (i + 1) / 2 + J + 1;
    I = i + J + 1;
}

// Lane K of each 16-lane row, broadcast to the whole row (DPP row_newbcast).
// In the diagonal-tile wave the four rows hold identical copies, so every lane
// receives lane K's value, and it arrives in a VGPR: read-lanes would route
// each broadcast through SGPRs, which run out when many broadcasts are live.
template <int K>
__device__ __forceinline__ double row_bcast(double v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xF, 0xF, true);
}

// Pivot step J of the right-looking Cholesky of a 16 x 16 diagonal tile.
// Lane i (i = lane % 16) holds row i of the partly reduced tile in a[] and
// column i of L^{-1} in x[] (the forward substitution L y = e_i, kept as its
// running right-hand side).  With d = A[J][J] and rr = 1/sqrt(d):
//   L[i][J] = A[i][J] rr on every lane, so lane k's value is L[k][J];
//   A[i][k] -= L[i][J] L[k][J]   for k > J   (trailing update of row i);
//   y[J] = w[J] rr, w[k] -= L[k][J] y[J]   for k > J   (substitution step).
// Only the pivot's reciprocal square root is serial; the 2 (15 - J) updates
// are independent of each other.
// acc += (lane K's src, broadcast to its 16-lane row) * mul in one
// instruction: the FP64 FMA with a DPP row_newbcast operand.  The same
// product and rounding as an FMA after a separate broadcast, one instruction
// instead of two.  Volatile, so the sequence keeps its order: NOP puts the two
// wait states a DPP read needs after a vector write of its source (the
// source of a step's first update is computed just before it).
template <int K, bool NOP>
__device__ __forceinline__ void fmac_bcast(double &acc, double src, double mul)
{
    if constexpr (NOP)
        asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc) : "v"(src), "v"(mul), "i"(K));
    else
        asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc) : "v"(src), "v"(mul), "i"(K));
}

template <int J, int K>
__device__ __forceinline__ void pivot_update(double (&a)[16], double (&x)[16], double lij, double nlij,
                                             double nyj)
{
    if constexpr (K > J) {
        // a[K] -= lij L[K][J] and x[K] -= L[K][J] yj, L[K][J] = lane K's lij
        fmac_bcast<K, K == J + 1>(a[K], lij, nlij);
        fmac_bcast<K, false>(x[K], lij, nyj);
    }
}

template <int J, int... K>
__device__ __forceinline__ void pivot_updates(double (&a)[16], double (&x)[16], double lij, double yj,
                                              std::integer_sequence<int, K...>)
{
    const double nlij = -lij, nyj = -yj;
    (pivot_update<J, K>(a, x, lij, nlij, nyj), ...);
    // two wait states before the next step's broadcast of a value written
    // by this step's last update
    asm volatile("s_nop 1");
}

template <int J>
__device__ __forceinline__ void pivot_step(double (&a)[16], double (&x)[16], double &mydiag, bool &bad,
                                           int ii)
{
    const double d = row_bcast<J>(a[J]);
    bad = bad || !(d > 0.0);
    // 1/sqrt(d): hardware estimate refined by two Newton steps
    // r <- r (3 - d r^2) / 2 (quadratic convergence: full FP64 from ~23
    // bits), then L_JJ = d r; no correctly rounded divide or square root on
    // this serial path.  A non-positive pivot continues as 1 (flagged).
    const double dd = d > 0.0 ? d : 1.0;
    double rr = __builtin_amdgcn_rsq(dd);
    rr = rr * (1.5 - 0.5 * dd * rr * rr);
    rr = rr * (1.5 - 0.5 * dd * rr * rr);
    const double gj = dd * rr;
    const double lij = a[J] * rr;
    const double yj = x[J] * rr;
    x[J] = yj;
    pivot_updates<J>(a, x, lij, yj, std::make_integer_sequence<int, 16>{});
    a[J] = (ii == J) ? gj : lij;
    mydiag = (ii == J) ? gj : mydiag;
}

template <int... J>
__device__ __forceinline__ void pivot_steps(double (&a)[16], double (&x)[16], double &mydiag, bool &bad,
                                            int ii, std::integer_sequence<int, J...>)
{
    (pivot_step<J>(a, x, mydiag, bad, ii), ...);
}

// Cholesky of one 16 x 16 diagonal tile (column-major in LDS) by one wave.
// The tile is overwritten with the inverse of its lower factor, the factor's
// diagonal goes to diag[0..15], and if g is given the factor's rows (global
// rows row0 + i < m) go to the packed lower store.  Returns true if a pivot
// was not positive (the factorization then continues with pivot 1, so every
// value stays finite).
__device__ __forceinline__ bool diag_factor(double *T, double *diag, double *g, int row0, int m)
{
    const int lane = threadIdx.x & 63;
    const int ii = lane & 15;
    double a[16], x[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        a[c] = T[c * TLD + ii];
        x[c] = (c == ii) ? 1.0 : 0.0;
    }
    double mydiag = 1.0;
    bool bad = false;
    pivot_steps(a, x, mydiag, bad, ii, std::make_integer_sequence<int, 16>{});
    // Only lanes 0-15 store the inverse.  This empty asm gives its values a
    // use on every lane, so the compiler cannot sink the substitution out of
    // the pivot steps into that conditional store, which would keep all 120
    // broadcasts live until then.
#pragma unroll
    for (int k = 0; k < 16; ++k)
        asm volatile("" : "+v"(x[k]));
    if (g && lane < 16) {
        const int i = row0 + ii;
        if (i < m) {
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c <= ii)
                    g[tri(i) + row0 + c] = a[c];
        }
    }
    if (lane < 16) {
        diag[ii] = mydiag;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            T[ii * TLD + i] = (i >= ii) ? x[i] : 0.0;
    }
    return bad;
}

// acc += op(A) * B with A in LDS (op = identity or transpose) and B a tile
// held in registers in the MFMA result layout (element t = row q + 4t),
// which is exactly the B-operand layout of the K-slice t.  NEG subtracts.
template <bool TA, bool NEG, int LDA = TLD>
__device__ __forceinline__ d4 tile_mma_rb(const double *A, const d4 B, d4 acc)
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const int k = q + 4 * kb;
        const double a = TA ? A[r * LDA + k] : A[k * LDA + r];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[kb], acc, 0, 0, NEG ? MFMA_NEG_A : 0);
    }
    return acc;
}

// The A operands of a tile for the four K-slices (op = identity or
// transpose), and the product with them already in registers: loading the
// next tile's operands before the current tile's four MFMAs keeps the LDS
// latency off the chain of dependent products.
template <bool TA>
__device__ __forceinline__ void tile_a(const double *A, double (&a)[4])
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const int k = q + 4 * kb;
        a[kb] = TA ? A[r * TLD + k] : A[k * TLD + r];
    }
}

template <bool NEG>
__device__ __forceinline__ d4 mma_a(const double (&a)[4], const d4 B, d4 acc)
{
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kb], B[kb], acc, 0, 0, NEG ? MFMA_NEG_A : 0);
    return acc;
}

// Step J of the forward substitution on a full leaf, operands one tile ahead:
// X[J] = L_JJ^{-1} X[J], then X[I] -= L_IJ X[J] for I > J.
template <int J>
__device__ __forceinline__ void fwd_step_full(d4 (&X)[NT_MAX], const double *Gt)
{
    double a[4], an[4];
    tile_a<false>(Gt + tix(J, J) * TSZ, a);
    if constexpr (J + 1 < NT_MAX)
        tile_a<false>(Gt + tix(J + 1, J) * TSZ, an);
    const d4 z = {0.0, 0.0, 0.0, 0.0};
    X[J] = mma_a<false>(a, X[J], z);
#pragma unroll
    for (int I = J + 1; I < NT_MAX; ++I) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
            a[kb] = an[kb];
        if (I + 1 < NT_MAX)
            tile_a<false>(Gt + tix(I + 1, J) * TSZ, an);
        X[I] = mma_a<true>(a, X[J], X[I]);
    }
}

// The backward substitution L^T z = y on a full leaf as one flat sequence of
// 36 tile products (for J = 7 .. 0: the diagonal block, then the blocks
// (J, I), I < J), each tile's operands loaded one product ahead.
__host__ __device__ constexpr int bwd_J(int t)
{
    int J = NT_MAX - 1;
    while (t > J) {
        t -= J + 1;
        --J;
    }
    return J;
}
__host__ __device__ constexpr int bwd_I(int t)   // -1: the diagonal block
{
    int J = NT_MAX - 1;
    while (t > J) {
        t -= J + 1;
        --J;
    }
    return t - 1;
}

template <int T>
__device__ __forceinline__ void bwd_task(d4 (&X)[NT_MAX], const double *Gt, double (&a)[4],
                                         double (&an)[4])
{
    constexpr int NTASK = NT_MAX * (NT_MAX + 1) / 2;
    constexpr int J = bwd_J(T), I = bwd_I(T);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
        a[kb] = an[kb];
    if constexpr (T + 1 < NTASK) {
        constexpr int J1 = bwd_J(T + 1), I1 = bwd_I(T + 1);
        tile_a<true>(Gt + tix(J1, I1 < 0 ? J1 : I1) * TSZ, an);
    }
    if constexpr (I < 0) {
        const d4 z = {0.0, 0.0, 0.0, 0.0};
        X[J] = mma_a<false>(a, X[J], z);
    } else {
        X[I] = mma_a<true>(a, X[J], X[I]);
    }
}

template <int... T>
__device__ __forceinline__ void bwd_tasks(d4 (&X)[NT_MAX], const double *Gt, double (&a)[4],
                                          double (&an)[4], std::integer_sequence<int, T...>)
{
    (bwd_task<T>(X, Gt, a, an), ...);
}

__device__ __forceinline__ void bwd_all_full(d4 (&X)[NT_MAX], const double *Gt)
{
    double a[4], an[4];
    tile_a<true>(Gt + tix(NT_MAX - 1, NT_MAX - 1) * TSZ, an);
    bwd_tasks(X, Gt, a, an, std::make_integer_sequence<int, NT_MAX * (NT_MAX + 1) / 2>{});
}

// Step J of the forward substitution L y = x on 16 columns held in registers
// (row tile I of the group in X[I], MFMA result layout): y_J = L_JJ^{-1} x_J,
// then x_I -= L_IJ y_J for I > J.  Gt holds L_JJ^{-1} in the diagonal slots.
// FULL: all NT_MAX row tiles present, so the tile updates carry no run-time
// condition and their LDS reads can be issued ahead of the products.
template <int J, bool FULL>
__device__ __forceinline__ void fwd_step(d4 (&X)[NT_MAX], const double *Gt, int nt)
{
    const d4 z = {0.0, 0.0, 0.0, 0.0};
    X[J] = tile_mma_rb<false, false>(Gt + tix(J, J) * TSZ, X[J], z);
#pragma unroll
    for (int I = J + 1; I < NT_MAX; ++I)
        if (FULL || I < nt)
            X[I] = tile_mma_rb<false, true>(Gt + tix(I, J) * TSZ, X[J], X[I]);
}

// the same for a run-time J (uniform): a switch, so that X stays in registers
template <bool FULL>
__device__ __forceinline__ void fwd_step_sw(int J, d4 (&X)[NT_MAX], const double *Gt, int nt)
{
    static_assert(NT_MAX == 8, "one case per row tile");
    switch (J) {
    case 0: fwd_step<0, FULL>(X, Gt, nt); break;
    case 1: fwd_step<1, FULL>(X, Gt, nt); break;
    case 2: fwd_step<2, FULL>(X, Gt, nt); break;
    case 3: fwd_step<3, FULL>(X, Gt, nt); break;
    case 4: fwd_step<4, FULL>(X, Gt, nt); break;
    case 5: fwd_step<5, FULL>(X, Gt, nt); break;
    case 6: fwd_step<6, FULL>(X, Gt, nt); break;
    case 7: fwd_step<7, FULL>(X, Gt, nt); break;
    default: break;
    }
}

__device__ __forceinline__ void fwd_step_rt(int J, d4 (&X)[NT_MAX], const double *Gt, int nt)
{
    if (nt == NT_MAX) {
        static_assert(NT_MAX == 8, "one case per row tile");
        switch (J) {
        case 0: fwd_step_full<0>(X, Gt); break;
        case 1: fwd_step_full<1>(X, Gt); break;
        case 2: fwd_step_full<2>(X, Gt); break;
        case 3: fwd_step_full<3>(X, Gt); break;
        case 4: fwd_step_full<4>(X, Gt); break;
        case 5: fwd_step_full<5>(X, Gt); break;
        case 6: fwd_step_full<6>(X, Gt); break;
        case 7: fwd_step_full<7>(X, Gt); break;
        default: break;
        }
    } else {
        fwd_step_sw<false>(J, X, Gt, nt);
    }
}

// backward substitution L^T z = y on the same register tiles
template <bool FULL>
__device__ __forceinline__ void bwd_all_t(d4 (&X)[NT_MAX], const double *Gt, int nt)
{
#pragma unroll
    for (int J = NT_MAX - 1; J >= 0; --J) {
        if (FULL || J < nt) {
            const d4 z = {0.0, 0.0, 0.0, 0.0};
            X[J] = tile_mma_rb<true, false>(Gt + tix(J, J) * TSZ, X[J], z);
#pragma unroll
            for (int I = 0; I < J; ++I)
                X[I] = tile_mma_rb<true, true>(Gt + tix(J, I) * TSZ, X[J], X[I]);
        }
    }
}

__device__ __forceinline__ void bwd_all(d4 (&X)[NT_MAX], const double *Gt, int nt)
{
    if (nt == NT_MAX)
        bwd_all_full(X, Gt);
    else
        bwd_all_t<false>(X, Gt, nt);
}

// columns [c0, c0 + 16) of the list (column 0 = the right-hand side y,
// others basis columns of W) on the leaf's rows into register tiles, lane
// (r, q) holding column c0 + r, rows 16 I + q + 4 t; missing entries are 0.
// A full leaf (every row inside) loads without conditions: lanes past the
// group read column 0 of W at the leaf's rows and zero the values after all
// loads are issued (an empty asm pins them, so that the zeroing stays a
// select and not one branch per load).
__device__ __forceinline__ void rhs_load(d4 (&X)[NT_MAX], const LeafArgs &A, int c0,
                                         const double *ysrc, const double *Wsrc, int64_t s,
                                         int64_t n, int nt, int m)
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const int nb = min(16, A.ncols - c0);
    const double *src = nullptr;
    if (r < nb) {
        const int col = A.cols[c0 + r];
        src = (col == 0) ? ysrc + s : Wsrc + (int64_t)col * n + s;
    }
    if (m == 16 * NT_MAX) {
        const double *p = src ? src : Wsrc + s;
#pragma unroll
        for (int I = 0; I < NT_MAX; ++I)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                X[I][t] = p[16 * I + q + 4 * t];
        if (nb < 16) {
#pragma unroll
            for (int I = 0; I < NT_MAX; ++I)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    asm volatile("" : "+v"(X[I][t]));
                    X[I][t] = src ? X[I][t] : 0.0;
                }
        }
        return;
    }
#pragma unroll
    for (int I = 0; I < NT_MAX; ++I)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int i = 16 * I + q + 4 * t;
            X[I][t] = (src && I < nt && i < m) ? src[i] : 0.0;
        }
}

template <typename PT>
__device__ __forceinline__ void rhs_store(const d4 (&X)[NT_MAX], const LeafArgs &A, int c0,
                                          PT *Xdst, int64_t s, int64_t n, int nt, int m)
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const int nb = min(16, A.ncols - c0);
    if (r < nb) {
        PT *dst = Xdst + (int64_t)A.cols[c0 + r] * n + s;
        if (m == 16 * NT_MAX) {   // full leaf: every row inside
#pragma unroll
            for (int I = 0; I < NT_MAX; ++I)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    dst[16 * I + q + 4 * t] = (PT)X[I][t];
            return;
        }
#pragma unroll
        for (int I = 0; I < NT_MAX; ++I)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = 16 * I + q + 4 * t;
                if (I < nt && i < m)
                    dst[i] = (PT)X[I][t];
            }
    }
}

template <typename PT>
__global__ __launch_bounds__(LEAF_MT, 2) void leaf_factor_kernel(LeafArgs A)
{
    __shared__ double Gt[NTRI * TSZ];   // lower factor tiles; diagonal slots hold L_JJ^{-1}
    __shared__ double s_diag[LEAF_LDS_MAX];   // diagonal of the factor
    __shared__ double s_red[LEAF_MW];
    __shared__ int s_bad;
    // the wave index is uniform in a wave: in a scalar register, the loops and
    // branches on it are scalar too
    const int tid = threadIdx.x, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63, r = l & 15, q = l >> 4;
    const int it = blockIdx.z;   // batch item
    const KParams kp = item_kp(A.kp, A.B, it);
    const double *__restrict__ Wsrc = ioff(A.W, A.B, it);
    PT *__restrict__ Xdst = ioff((PT *)A.Xt, A.B, it);
    double *leaf_ld = ioff(A.leaf_ld, A.B, it);
    int *status = ioff(A.status, A.B, it);
    const double *ysrc = A.y ? A.y + it * A.B.ystride : nullptr;
    const int64_t b = blockIdx.x;
    const int64_t h = A.leaf0 + b;
    const int64_t s = A.start[h];
    const int m = (int)(A.end[h] - s);
    const int64_t n = A.n;
    if (m == 0) {
        if (tid == 0)
            leaf_ld[b] = 0.0;
        return;
    }
    const int nt = (m + 15) >> 4;
    double *gout = A.G ? A.G + b * A.gstride : nullptr;
    // C_lambda^{-1} is applied to the column list in groups of 16 columns, one
    // group per wave, held in registers.  Groups 0..2 belong to waves 1..3
    // from the start: their loads are in flight during the evaluation (issued
    // after the evaluation's own global loads have returned: the wait on
    // those would otherwise include them), and their forward substitution
    // runs inside the factorization (step J once L_JJ^{-1} and column J of L
    // exist), in the time those waves would otherwise wait for wave 0's
    // serial diagonal factorizations; only the backward substitution is left
    // after it.
    const int ngrp = (A.ncols - A.cbeg + 15) / 16;
    const int pg = wid - 1;
    const bool piped = wid > 0 && pg < ngrp;
    d4 X[NT_MAX];
    bool bad = false;   // wave 0 only
    // Separable form for 1-D exponential-family kernels on an ascending leaf:
    // for x_i >= x_k, exp(-c (x_i - x_k)) = E_i F_k with E_i = exp(-c (x_i -
    // x_0)) and F_k = exp(c (x_k - x_0)), x_0 the leaf's first point, so the
    // leaf takes 2 m exponentials instead of one exponential and one square
    // root per entry.  Used when the leaf is checked to be in ascending order
    // and c times its span is below 500 (every factor far inside the FP64
    // range); the entries then differ from direct evaluation by a few units
    // in the last place, and the diagonal is exactly a^2 + sigma^2 (plus the
    // point's own variance when per-point noise is given).  E, F and the
    // points pass through LDS words the tiles never use (the 17th entry of
    // each tile column); every thread then holds the factors of its 8 rows
    // and 8 columns, and an entry of a tile below the diagonal block row
    // costs three multiplies and a subtraction.
    const bool sep_kind = kp.dim == 1 && (kp.kind == HODLR_K_MATERN32 || kp.kind == HODLR_K_EXP);
    bool sep = false;
    if (sep_kind) {
        static_assert(3 * LEAF_LDS_MAX <= NTRI * 16, "padding words for E, F and the points");
        auto pad = [&](int j) -> double & { return Gt[(j >> 4) * TSZ + (j & 15) * TLD + 16]; };
        const int i = tid & (LEAF_LDS_MAX - 1);
        const double x0 = A.x[s], xl = A.x[s + m - 1];
        const double xi = i < m ? A.x[s + i] : 0.0;
        const double xn = tid + 1 < m ? A.x[s + tid + 1] : 0.0;   // tid + 1 < m implies tid < 128
        const int unsorted = (tid + 1 < m && xn < xi) ? 1 : 0;
        sep = !__syncthreads_or(unsorted) && kp.c * (xl - x0) < 500.0;
        if (sep) {
            if (i < m) {
                pad(tid) = exp((tid < LEAF_LDS_MAX ? -kp.c : kp.c) * (xi - x0));   // E then F
                if (tid < LEAF_LDS_MAX)
                    pad(2 * LEAF_LDS_MAX + i) = xi;
            }
            __syncthreads();
            static_assert(LEAF_MT == 256, "one tile element per thread");
            const int rr = tid & 15, cc = tid >> 4;
            double aE[NT_MAX], xr1[NT_MAX], Fc[NT_MAX], xc1[NT_MAX];
#pragma unroll
            for (int I = 0; I < NT_MAX; ++I) {
                const int ic = min(16 * I + rr, m - 1), kc = min(16 * I + cc, m - 1);
                aE[I] = kp.a2 * pad(ic);
                xr1[I] = pad(2 * LEAF_LDS_MAX + ic);
                Fc[I] = pad(LEAF_LDS_MAX + kc);
                xc1[I] = pad(2 * LEAF_LDS_MAX + kc);
            }
            const bool matern = kp.kind == HODLR_K_MATERN32;
            const double dg = kp.a2 + kp.sigma2;
#pragma unroll
            for (int I = 0; I < NT_MAX; ++I) {
#pragma unroll
                for (int K = 0; K <= I; ++K) {
                    if (I < nt) {
                        double v;
                        if (K < I && 16 * I + 15 < m) {
                            // below the diagonal block row, every row inside the leaf
                            const double e = aE[I] * Fc[K];
                            v = matern ? e * (1.0 + kp.c * (xr1[I] - xc1[K])) : e;
                        } else if (K == I && 16 * I + 15 < m) {
                            // a diagonal block inside the leaf: selects only
                            const int ii = 16 * I + rr, k = 16 * K + cc;
                            const double e = aE[I] * Fc[K];
                            const double off = matern ? e * (1.0 + kp.c * (xr1[I] - xc1[K])) : e;
                            const double nz = kp.noise ? kp.noise[s + ii] : 0.0;
                            v = ii > k ? off : (ii == k ? dg + nz : 0.0);
                        } else {
                            const int ii = 16 * I + rr, k = 16 * K + cc;
                            if (ii < m && k < m) {
                                const double e = aE[I] * Fc[K];
                                const double off = matern ? e * (1.0 + kp.c * (xr1[I] - xc1[K])) : e;
                                v = ii > k ? off
                                           : (ii == k ? dg + (kp.noise ? kp.noise[s + ii] : 0.0) : 0.0);
                            } else {
                                v = (ii == k) ? 1.0 : 0.0;
                            }
                        }
                        Gt[tix(I, K) * TSZ + cc * TLD + rr] = v;
                    }
                }
            }
        }
    }
    if (!sep) {
        // C = K + sigma^2 I on the lower tiles, identity on the padding.
        // With 256 threads every thread owns the same element (rr, cc) of
        // each tile, so it needs only 8 row and 8 column points.
        static_assert(LEAF_MT == 256, "one tile element per thread");
        const int rr = tid & 15, cc = tid >> 4;
        double xr[3][NT_MAX], xk[3][NT_MAX];
#pragma unroll
        for (int I = 0; I < NT_MAX; ++I) {
            int i = 16 * I + rr, k = 16 * I + cc;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                xr[d][I] = (d < kp.dim && i < m) ? A.x[d * n + s + i] : 0.0;
                xk[d][I] = (d < kp.dim && k < m) ? A.x[d * n + s + k] : 0.0;
            }
        }
        // entries above the diagonal of a diagonal tile are never read by
        // the factorization (it works on the lower triangle) and are left zero
#pragma unroll
        for (int I = 0; I < NT_MAX; ++I) {
#pragma unroll
            for (int K = 0; K <= I; ++K) {
                if (I < nt) {
                    const int i = 16 * I + rr, k = 16 * K + cc;
                    double v;
                    if (i < m && k < m && i >= k) {
                        double r2 = 0.0;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            double t = xr[d][I] - xk[d][K];
                            r2 += t * t;
                        }
                        v = kfun_r2<double>(kp.kind, kp.a2, kp.c, r2);
                        if (i == k)
                            v += kp.sigma2 + (kp.noise ? kp.noise[s + i] : 0.0);
                    } else {
                        v = (i == k) ? 1.0 : 0.0;
                    }
                    Gt[tix(I, K) * TSZ + cc * TLD + rr] = v;
                }
            }
        }
    }
    __syncthreads();
    if (piped)
        rhs_load(X, A, A.cbeg + 16 * pg, ysrc, Wsrc, s, n, nt, m);
    if (wid == 0)
        bad = diag_factor(Gt, s_diag, gout, 0, m);
    __syncthreads();
    for (int J = 0; J < nt; ++J) {
        // panel: L_IJ = C_IJ L_JJ^{-T}, two tiles per wave at most (8 row tiles)
        {
            static_assert(NT_MAX <= 1 + 2 * LEAF_MW, "panel tiles per wave");
            const int I1 = J + 1 + wid, I2 = I1 + LEAF_MW;
            const double *D = Gt + tix(J, J) * TSZ;
            if (I2 < nt)
                tile_panel2<true>(Gt + tix(I1, J) * TSZ, Gt + tix(I2, J) * TSZ, D);
            else if (I1 < nt)
                tile_panel2<false>(Gt + tix(I1, J) * TSZ, nullptr, D);
        }
        __syncthreads();
        if (J + 1 < nt) {
            // wave 0: next diagonal tile first (look-ahead), then factor it
            if (wid == 0) {
                double *T = Gt + tix(J + 1, J + 1) * TSZ;
                const double *P = Gt + tix(J + 1, J) * TSZ;
                d4 acc = {0.0, 0.0, 0.0, 0.0};
                acc = tile_mma<false>(P, P, acc);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    T[r * TLD + q + 4 * t] -= acc[t];
                bad = diag_factor(T, s_diag + 16 * (J + 1), gout, 16 * (J + 1), m) || bad;
            }
            // remaining trailing tiles C_IK -= L_IJ L_KJ^T (J < K <= I): the
            // first ones on the other three waves (which also run their
            // forward substitution step), and while there are many, the last
            // (ntask - 8) / 3 on wave 0 after its diagonal factorization
            // (the balance point measured per step)
            const int Tn = nt - 1 - J;
            const int ntask = Tn * (Tn + 1) / 2 - 1;
            const int n0 = ntask > 8 ? (ntask - 8) / 3 : 0;
            const int t0 = wid == 0 ? ntask - n0 : wid - 1;
            const int t1 = wid == 0 ? ntask : ntask - n0;
            const int ts = wid == 0 ? 1 : LEAF_MW - 1;
            // two tasks at a time, their products interleaved
            for (int task = t0; task < t1; task += 2 * ts) {
                int I1, K1;
                trail_tile(task, J, I1, K1);
                if (task + ts < t1) {
                    int I2, K2;
                    trail_tile(task + ts, J, I2, K2);
                    tile_sub2<true>(Gt + tix(I1, K1) * TSZ, Gt + tix(I1, J) * TSZ, Gt + tix(K1, J) * TSZ,
                                    Gt + tix(I2, K2) * TSZ, Gt + tix(I2, J) * TSZ, Gt + tix(K2, J) * TSZ);
                } else {
                    tile_sub2<false>(Gt + tix(I1, K1) * TSZ, Gt + tix(I1, J) * TSZ, Gt + tix(K1, J) * TSZ,
                                     nullptr, nullptr, nullptr);
                }
            }
        }
        if (piped)
            fwd_step_rt(J, X, Gt, nt);
        __syncthreads();
    }
    // log det of the leaf, 2 sum_i log L_ii over its real rows: one log per
    // thread, off the serial path of the factorization
    double lgp = 0.0;
    if (tid < m)
        lgp = log(s_diag[tid]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        lgp += __shfl_xor(lgp, o, 64);
    if (l == 0)
        s_red[wid] = lgp;
    if (tid == 0)
        s_bad = bad ? 1 : 0;
    __syncthreads();
    double lg = 0.0;
#pragma unroll
    for (int w = 0; w < LEAF_MW; ++w)
        lg += s_red[w];
    if (s_bad || !(lg == lg)) {
        if (tid == 0) {
            atomicOr(status, DS_NOTSPD_LEAF);
            leaf_ld[b] = __builtin_nan("");
        }
        return;
    }
    if (tid == 0)
        leaf_ld[b] = 2.0 * lg;
    if (gout) {   // off-diagonal factor tiles (the diagonal ones went out in diag_factor)
        for (int idx = tid; idx < tri(m); idx += LEAF_MT) {
            int i = tri_row(idx), k = idx - tri(i);
            if ((i >> 4) != (k >> 4))
                gout[idx] = Gt[tix(i >> 4, k >> 4) * TSZ + (k & 15) * TLD + (i & 15)];
        }
    }
    if (piped) {
        bwd_all(X, Gt, nt);
        rhs_store(X, A, A.cbeg + 16 * pg, Xdst, s, n, nt, m);
    }
    // further groups: both substitutions here, round-robin over the waves.
    // Full groups of 16 issue the fewest MFMAs (42 columns: 16 + 16 + 10 on
    // three waves measured faster than 11 + 11 + 11 + 9 on four).
    for (int g = (LEAF_MW - 1) + wid; g < ngrp; g += LEAF_MW) {
        const int c0 = A.cbeg + 16 * g;
        rhs_load(X, A, c0, ysrc, Wsrc, s, n, nt, m);
#pragma unroll
        for (int J = 0; J < NT_MAX; ++J)
            if (J < nt)
                fwd_step_rt(J, X, Gt, nt);
        bwd_all(X, Gt, nt);
        rhs_store(X, A, c0, Xdst, s, n, nt, m);
    }
}

// ---------------------------------------------------------------------------
// Leaves of LEAF_LDS_MAX + 1 .. LEAF_MAX points.  Their lower triangle (up to
// 136 tiles) does not fit one CU's LDS, so the leaf is factored as the 2 x 2
// block matrix [[C11, .], [C21, C22]], C11 its first 128 rows:
//   C11 = L11 L11^T in LDS;
//   L21 = C21 L11^{-T}: each wave evaluates tile rows of C21^T on the fly into
//         registers, solves them with L11 and stores them in HBM (16 x 16
//         tiles, column-major), where they stay for the right-hand sides;
//   S = C22 - L21 L21^T in LDS, then S = L22 L22^T.
// The right-hand sides go through L11, L21 and L22 (forward), then L22^T,
// L21^T and L11^T (backward), 16 columns per wave in registers.
constexpr int L21_TSZ = 256;                      // doubles per HBM tile
constexpr int L21_TILES = NT_MAX * NT_MAX;        // tiles per leaf
constexpr size_t L21_LEAF = (size_t)L21_TILES * L21_TSZ;

// Blocked right-looking Cholesky of the nt x nt lower tiles at Gt: wave 0
// factors the diagonal tiles (with look-ahead), all waves the panels and the
// trailing tiles.  Tile 0 starts at row and column g0 of the leaf (for the
// packed store and the diagonal).  Returns wave 0's non-positive-pivot flag.
__device__ bool factor_tiles(double *Gt, double *diag, double *gout, int g0, int nt, int m)
{
    // the wave index is uniform in a wave: in a scalar register, the loops and
    // branches on it are scalar too
    const int tid = threadIdx.x, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63, r = l & 15, q = l >> 4;
    bool bad = false;
    if (wid == 0)
        bad = diag_factor(Gt, diag, gout, g0, m);
    __syncthreads();
    for (int J = 0; J < nt; ++J) {
        for (int I = J + 1 + wid; I < nt; I += LEAF_MW) {
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            double *T = Gt + tix(I, J) * TSZ;
            acc = tile_mma<false>(T, Gt + tix(J, J) * TSZ, acc);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                T[r * TLD + q + 4 * t] = acc[t];
        }
        __syncthreads();
        if (J + 1 < nt) {
            if (wid == 0) {
                double *T = Gt + tix(J + 1, J + 1) * TSZ;
                const double *P = Gt + tix(J + 1, J) * TSZ;
                d4 acc = {0.0, 0.0, 0.0, 0.0};
                acc = tile_mma<false>(P, P, acc);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    T[r * TLD + q + 4 * t] -= acc[t];
                bad = diag_factor(T, diag + 16 * (J + 1), gout, g0 + 16 * (J + 1), m) || bad;
            }
            const int Tn = nt - 1 - J;
            const int ntask = Tn * (Tn + 1) / 2 - 1;
            const int n0 = ntask > 8 ? (ntask - 8) / 3 : 0;
            const int t0 = wid == 0 ? ntask - n0 : wid - 1;
            const int t1 = wid == 0 ? ntask : ntask - n0;
            const int ts = wid == 0 ? 1 : LEAF_MW - 1;
            for (int task = t0; task < t1; task += ts) {
                int tt = task + 1;   // skip the look-ahead tile (I = K = J+1)
                int I = 0;
                while ((I + 1) * (I + 2) / 2 <= tt)
                    ++I;
                int K = tt - I * (I + 1) / 2;
                I += J + 1;
                K += J + 1;
                d4 acc = {0.0, 0.0, 0.0, 0.0};
                acc = tile_mma<false>(Gt + tix(I, J) * TSZ, Gt + tix(K, J) * TSZ, acc);
                double *T = Gt + tix(I, K) * TSZ;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    T[r * TLD + q + 4 * t] -= acc[t];
            }
        }
        __syncthreads();
    }
    return bad;
}

// C + sigma^2 I on the lower tiles of rows [off, off + mm) of the leaf (tile
// rows and columns of that range only), identity on the padding
__device__ void eval_region(double *Gt, const KParams &kp, const double *__restrict__ x, int64_t n,
                            int64_t s, int off, int mm)
{
    const int tid = threadIdx.x;
    const int nt = (mm + 15) >> 4;
    const int rr = tid & 15, cc = tid >> 4;
    double xr[3][NT_MAX], xk[3][NT_MAX];
#pragma unroll
    for (int I = 0; I < NT_MAX; ++I) {
        const int i = 16 * I + rr, k = 16 * I + cc;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xr[d][I] = (d < kp.dim && i < mm) ? x[d * n + s + off + i] : 0.0;
            xk[d][I] = (d < kp.dim && k < mm) ? x[d * n + s + off + k] : 0.0;
        }
    }
#pragma unroll
    for (int I = 0; I < NT_MAX; ++I) {
#pragma unroll
        for (int K = 0; K <= I; ++K) {
            if (I < nt) {
                const int i = 16 * I + rr, k = 16 * K + cc;
                double v;
                if (i < mm && k < mm && i >= k) {
                    double r2 = 0.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const double t = xr[d][I] - xk[d][K];
                        r2 += t * t;
                    }
                    v = kfun_r2<double>(kp.kind, kp.a2, kp.c, r2);
                    if (i == k)
                        v += kp.sigma2 + (kp.noise ? kp.noise[s + off + i] : 0.0);
                } else {
                    v = (i == k) ? 1.0 : 0.0;
                }
                Gt[tix(I, K) * TSZ + cc * TLD + rr] = v;
            }
        }
    }
}

template <typename PT>
__global__ __launch_bounds__(LEAF_MT, 1) void leaf_factor_big_kernel(LeafArgs A)
{
    __shared__ double G1[NTRI * TSZ];   // L11 tiles (diagonal slots: L_JJ^{-1})
    __shared__ double G2[NTRI * TSZ];   // C22, then S, then L22 tiles
    __shared__ double s_diag[LEAF_MAX];
    __shared__ double s_red[LEAF_MW];
    __shared__ int s_bad;
    static_assert(LEAF_MAX == 2 * LEAF_LDS_MAX && LEAF_MT == LEAF_MAX, "two halves, a thread per row");
    // the wave index is uniform in a wave: in a scalar register, the loops and
    // branches on it are scalar too
    const int tid = threadIdx.x, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63, r = l & 15, q = l >> 4;
    const int it = blockIdx.z;   // batch item
    const KParams kp = item_kp(A.kp, A.B, it);
    const double *__restrict__ Wsrc = ioff(A.W, A.B, it);
    PT *__restrict__ Xdst = ioff((PT *)A.Xt, A.B, it);
    double *leaf_ld = ioff(A.leaf_ld, A.B, it);
    int *status = ioff(A.status, A.B, it);
    const double *ysrc = A.y ? A.y + it * A.B.ystride : nullptr;
    const int64_t b = blockIdx.x;
    const int64_t h = A.leaf0 + b;
    const int64_t s = A.start[h];
    const int m = (int)(A.end[h] - s);
    const int64_t n = A.n;
    double *L21 = ioff(A.L21, A.B, it) + b * (int64_t)L21_LEAF;
    if (m == 0) {
        if (tid == 0)
            leaf_ld[b] = 0.0;
        return;
    }
    const int m1 = m < LEAF_LDS_MAX ? m : LEAF_LDS_MAX, m2 = m - m1;
    const int nt1 = (m1 + 15) >> 4, nt2 = (m2 + 15) >> 4;
    double *gout = A.G ? A.G + b * A.gstride : nullptr;
    eval_region(G1, kp, A.x, n, s, 0, m1);
    if (m2 > 0)
        eval_region(G2, kp, A.x, n, s, m1, m2);
    __syncthreads();
    bool bad = factor_tiles(G1, s_diag, gout, 0, nt1, m);
    if (m2 > 0) {
        // L21 = C21 L11^{-T}, one tile row per wave: lane (r, q) holds entry
        // (16 J + q + 4 t, r) of C21^T, i.e. k(x_k, x_c) with k in the first
        // half and c = 128 + 16 I2 + r
        for (int I2 = wid; I2 < nt2; I2 += LEAF_MW) {
            const int pc = LEAF_LDS_MAX + 16 * I2 + r;
            const bool cok = pc < m;
            double xc[3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                xc[d] = (d < kp.dim && cok) ? A.x[d * n + s + pc] : 0.0;
            d4 X[NT_MAX];
#pragma unroll
            for (int J = 0; J < NT_MAX; ++J)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 16 * J + q + 4 * t;
                    double r2 = 0.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const double u = (d < kp.dim ? A.x[d * n + s + k] : 0.0) - xc[d];
                        r2 += u * u;
                    }
                    X[J][t] = cok ? kfun_r2<double>(kp.kind, kp.a2, kp.c, r2) : 0.0;
                }
#pragma unroll
            for (int J = 0; J < NT_MAX; ++J)
                fwd_step_rt(J, X, G1, NT_MAX);
            // tile (I2, J) of L21 is the transpose of register tile J
            double *dst = L21 + (int64_t)I2 * NT_MAX * L21_TSZ;
#pragma unroll
            for (int J = 0; J < NT_MAX; ++J)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    dst[J * L21_TSZ + (q + 4 * t) * 16 + r] = X[J][t];
        }
        __syncthreads();   // L21 written (work-group scope) before it is read
        // S = C22 - L21 L21^T on the lower tiles of the second half
        const int ntask = nt2 * (nt2 + 1) / 2;
        for (int task = wid; task < ntask; task += LEAF_MW) {
            int I = 0;
            while ((I + 1) * (I + 2) / 2 <= task)
                ++I;
            const int K = task - I * (I + 1) / 2;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int J = 0; J < NT_MAX; ++J)
                acc = tile_mma<false, 16, 16>(L21 + (int64_t)(I * NT_MAX + J) * L21_TSZ,
                                              L21 + (int64_t)(K * NT_MAX + J) * L21_TSZ, acc);
            double *T = G2 + tix(I, K) * TSZ;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                T[r * TLD + q + 4 * t] -= acc[t];
        }
        __syncthreads();
        bad = factor_tiles(G2, s_diag + LEAF_LDS_MAX, gout, LEAF_LDS_MAX, nt2, m) || bad;
    }
    double lgp = tid < m ? log(s_diag[tid]) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        lgp += __shfl_xor(lgp, o, 64);
    if (l == 0)
        s_red[wid] = lgp;
    if (tid == 0)
        s_bad = 0;
    __syncthreads();
    if (bad)
        s_bad = 1;   // wave 0 of each half's factorization
    __syncthreads();
    double lg = 0.0;
#pragma unroll
    for (int w = 0; w < LEAF_MW; ++w)
        lg += s_red[w];
    if (s_bad || !(lg == lg)) {
        if (tid == 0) {
            atomicOr(status, DS_NOTSPD_LEAF);
            leaf_ld[b] = __builtin_nan("");
        }
        return;
    }
    if (tid == 0)
        leaf_ld[b] = 2.0 * lg;
    if (gout) {   // the off-diagonal parts of the packed factor (diagonal tiles went out above)
        for (int idx = tid; idx < tri(m); idx += LEAF_MT) {
            const int i = tri_row(idx), k = idx - tri(i);
            if (i < LEAF_LDS_MAX) {
                if ((i >> 4) != (k >> 4))
                    gout[idx] = G1[tix(i >> 4, k >> 4) * TSZ + (k & 15) * TLD + (i & 15)];
            } else if (k < LEAF_LDS_MAX) {
                const int i2 = i - LEAF_LDS_MAX;
                gout[idx] = L21[(int64_t)((i2 >> 4) * NT_MAX + (k >> 4)) * L21_TSZ + (k & 15) * 16 +
                                (i2 & 15)];
            } else {
                const int i2 = i - LEAF_LDS_MAX, k2 = k - LEAF_LDS_MAX;
                if ((i2 >> 4) != (k2 >> 4))
                    gout[idx] = G2[tix(i2 >> 4, k2 >> 4) * TSZ + (k2 & 15) * TLD + (i2 & 15)];
            }
        }
    }
    // C_lambda^{-1} on the column list, 16 columns per wave
    const int ngrp = (A.ncols - A.cbeg + 15) / 16;
    for (int g = wid; g < ngrp; g += LEAF_MW) {
        const int c0 = A.cbeg + 16 * g;
        // the tile addresses are the same for every group: recomputed per
        // group rather than held across the loop (256 of them would spill)
        const double *Lg = L21;
        asm volatile("" : "+s"(Lg));
        d4 X1[NT_MAX], X2[NT_MAX];
        rhs_load(X1, A, c0, ysrc, Wsrc, s, n, nt1, m1);
        if (m2 > 0)
            rhs_load(X2, A, c0, ysrc, Wsrc, s + LEAF_LDS_MAX, n, nt2, m2);
#pragma unroll
        for (int J = 0; J < NT_MAX; ++J)
            if (J < nt1)
                fwd_step_rt(J, X1, G1, nt1);
        if (m2 > 0) {
#pragma unroll
            for (int I2 = 0; I2 < NT_MAX; ++I2)
                if (I2 < nt2)
#pragma unroll
                    for (int J = 0; J < NT_MAX; ++J)
                        X2[I2] = tile_mma_rb<false, true, 16>(
                            Lg + (int64_t)(I2 * NT_MAX + J) * L21_TSZ, X1[J], X2[I2]);
#pragma unroll
            for (int J = 0; J < NT_MAX; ++J)
                if (J < nt2)
                    fwd_step_rt(J, X2, G2, nt2);
            bwd_all(X2, G2, nt2);
#pragma unroll
            for (int J = 0; J < NT_MAX; ++J)
#pragma unroll
                for (int I2 = 0; I2 < NT_MAX; ++I2)
                    if (I2 < nt2)
                        X1[J] = tile_mma_rb<true, true, 16>(
                            Lg + (int64_t)(I2 * NT_MAX + J) * L21_TSZ, X2[I2], X1[J]);
        }
        bwd_all(X1, G1, nt1);
        rhs_store(X1, A, c0, Xdst, s, n, nt1, m1);
        if (m2 > 0)
            rhs_store(X2, A, c0, Xdst, s + LEAF_LDS_MAX, n, nt2, m2);
    }
}

// z <- C_lambda^{-1} z with the stored packed factor, for leaves above
// LEAF_LDS_MAX (the factor does not fit LDS): thread i owns row i; the
// forward sweep goes by columns of L (one broadcast per step), the backward
// one by rows of L (contiguous reads).
template <typename PT>
__global__ __launch_bounds__(LEAF_MT) void leaf_solve_big_kernel(LeafArgs A, PT *z)
{
    __shared__ double zs[LEAF_MAX];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t h = A.leaf0 + b;
    const int64_t s = A.start[h];
    const int m = (int)(A.end[h] - s);
    if (m == 0)
        return;
    const double *g = A.G + b * A.gstride;
    const bool in = tid < m;
    double v = in ? (double)z[s + tid] : 0.0;
    const double dii = in ? g[tri(tid) + tid] : 1.0;
    // L y = z
    for (int j = 0; j < m; ++j) {
        if (tid == j)
            zs[j] = v / dii;
        __syncthreads();
        if (tid > j && in)
            v -= g[tri(tid) + j] * zs[j];
    }
    __syncthreads();
    v = in ? zs[tid] : 0.0;
    // L^T x = y
    for (int j = m - 1; j >= 0; --j) {
        if (tid == j)
            zs[j] = v / dii;
        __syncthreads();
        if (tid < j)
            v -= g[tri(j) + tid] * zs[j];
    }
    __syncthreads();
    if (in)
        z[s + tid] = (PT)zs[tid];
}

// the value lane l (uniform) holds, in every lane
__device__ __forceinline__ double lane_value(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// z <- C_lambda^{-1} z on each leaf with the stored packed factors (row i of
// L at G[i (i + 1) / 2 ...]): one wave per leaf, the factor copied to LDS by
// direct global-to-LDS loads, lane l holding rows l and l + 64 of the vector.
// With D = diag(L) and the unit-diagonal L' = L D^{-1}:  L' v = z, then
// L'^T w = D^{-2} v gives w = C^{-1} z.  The forward sweep goes by columns of
// L' (step j reads L_ij down column j, whose packed addresses fall in distinct
// LDS banks for 32 consecutive rows), the backward one by rows of L
// (contiguous); each step broadcasts the finished entry from its lane, and the
// scaling by 1 / L_jj is applied to the read entries, off the dependency
// chain of the sweep.
template <typename PT>
__global__ __launch_bounds__(LEAF_SOLVE_T) void leaf_solve_kernel(LeafArgs A, PT *z)
{
    extern __shared__ double Lp[];
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t h = A.leaf0 + b;
    const int64_t s = A.start[h];
    const int m = (int)(A.end[h] - s);
    if (m == 0)
        return;
    const double *g = A.G + b * A.gstride;
    const int ntri = tri(m);
    // 1 KB per instruction (16 bytes a lane) when the leaf's factor starts on
    // 16 bytes, all issued before one wait; the rest by ordinary loads
    int base = 0;
    if (((uintptr_t)g & 15) == 0)
        for (; base + 2 * LEAF_SOLVE_T <= ntri; base += 2 * LEAF_SOLVE_T)
            __builtin_amdgcn_global_load_lds((const void *)(g + base + 2 * lane),
                                             (__attribute__((address_space(3))) void *)(Lp + base),
                                             16, 0, 0);
    for (; base + 8 * LEAF_SOLVE_T <= ntri; base += 8 * LEAF_SOLVE_T) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = g[base + u * LEAF_SOLVE_T + lane];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            Lp[base + u * LEAF_SOLVE_T + lane] = v[u];
    }
    for (int idx = base + lane; idx < ntri; idx += LEAF_SOLVE_T)
        Lp[idx] = g[idx];
    const int ra = lane, rb = lane + 64;
    const bool ina = ra < m, inb = rb < m;
    double xa = ina ? (double)z[s + ra] : 0.0;
    double xb = inb ? (double)z[s + rb] : 0.0;
    __builtin_amdgcn_s_waitcnt(0);   // the direct loads have landed in LDS
    __syncthreads();
    const int ta = tri(ra), tb = tri(rb);
    const double ia = ina ? 1.0 / Lp[ta + ra] : 0.0;
    const double ib = inb ? 1.0 / Lp[tb + rb] : 0.0;
    const int ma = min(m, 64);
    // Steps go in blocks of SB: the block's LDS entries are read and scaled
    // first (they do not depend on the broadcasts), then its steps run.  A
    // lane whose entry is not used takes 0 (its value is left as it is), so
    // every index read is below tri(m).
    constexpr int SB = 8;
    auto pick = [&](bool use, int idx) {   // an unconditional read, then a select
        const double v = Lp[use ? idx : 0];
        return use ? v : 0.0;
    };
    auto fa = [&](int j) { return pick(ra > j && ina, ta + j); };
    auto fb = [&](int j) { return pick(rb > j && inb, tb + j); };
    auto ga = [&](int j) { return pick(ra < j, tri(j) + ra); };
    auto gb = [&](int j) { return pick(rb < j, tri(j) + rb); };
    // L' v = z, by columns
    for (int j0 = 0; j0 < ma; j0 += SB) {
        double ca[SB], cb[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const double d = lane_value(ia, min(j0 + u, 63));
            ca[u] = fa(j0 + u) * d;
            cb[u] = fb(j0 + u) * d;
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int j = j0 + u;
            if (j < ma) {
                const double vj = lane_value(xa, j);
                xa = fma(-ca[u], vj, xa);
                xb = fma(-cb[u], vj, xb);
            }
        }
    }
    for (int j0 = 64; j0 < m; j0 += SB) {
        double cb[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u)
            cb[u] = fb(j0 + u) * lane_value(ib, min(j0 + u - 64, 63));
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int j = j0 + u;
            if (j < m) {
                const double vj = lane_value(xb, j - 64);
                xb = fma(-cb[u], vj, xb);
            }
        }
    }
    // L'^T w = D^{-2} v, by rows of L (row j of L scaled by 1 / L_ii in lane i)
    xa *= ia * ia;
    xb *= ib * ib;
    for (int j0 = m - 1; j0 >= 64; j0 -= SB) {
        double ca[SB], cb[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int j = max(j0 - u, 0);
            ca[u] = ga(j) * ia;
            cb[u] = gb(j) * ib;
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int j = j0 - u;
            if (j >= 64) {
                const double wj = lane_value(xb, j - 64);
                xb = fma(-cb[u], wj, xb);
                xa = fma(-ca[u], wj, xa);
            }
        }
    }
    for (int j0 = ma - 1; j0 >= 0; j0 -= SB) {
        double ca[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u)
            ca[u] = ga(max(j0 - u, 0)) * ia;
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int j = j0 - u;
            if (j >= 0) {
                const double wj = lane_value(xa, j);
                xa = fma(-ca[u], wj, xa);
            }
        }
    }
    if (ina)
        z[s + ra] = (PT)xa;
    if (inb)
        z[s + rb] = (PT)xb;
}

static LeafArgs leaf_args(Pipeline &P)
{
    const Plan &p = *P.plan;
    LeafArgs A;
    A.x = P.x;
    A.n = p.n;
    A.kp = P.kp;
    A.start = p.d_start;
    A.end = p.d_end;
    A.leaf0 = p.nint;
    A.W = wsp<double>(P, P.lay.W);
    A.Xt = P.ws + P.lay.Xt;
    A.y = nullptr;
    A.cols = wsp<int>(P, P.lay.cols);
    A.ncols = 0;
    A.cbeg = 1;
    A.G = P.lay.store_leaf ? wsp<double>(P, P.lay.G) : nullptr;
    A.gstride = (int64_t)p.leafmax * (p.leafmax + 1) / 2;
    A.leaf_ld = wsp<double>(P, P.lay.leaf_ld);
    A.status = wsp<int>(P, P.lay.status);
    A.L21 = wsp<double>(P, P.lay.L21);
    A.B = P.batch;
    return A;
}

void run_leaf_factor(Pipeline &P, const double *y)
{
    const Plan &p = *P.plan;
    if (p.leafmax > LEAF_MAX)
        throw Error{HODLR_EINVAL, "leaf size above 256 is not supported"};
    LeafArgs A = leaf_args(P);
    A.y = y;
    P.rhs = y;
    A.cbeg = y ? 0 : 1;
    A.ncols = P.cnt[p.L];
    ProfScope ps(P.stream, PS_LEAF);
    const dim3 grid((unsigned)p.nleaf, 1, P.nitems);
    if (p.leafmax > LEAF_LDS_MAX) {
        if (p.f32())
            leaf_factor_big_kernel<float><<<grid, LEAF_MT, 0, P.stream>>>(A);
        else
            leaf_factor_big_kernel<double><<<grid, LEAF_MT, 0, P.stream>>>(A);
    } else if (p.f32()) {
        leaf_factor_kernel<float><<<grid, LEAF_MT, 0, P.stream>>>(A);
    } else {
        leaf_factor_kernel<double><<<grid, LEAF_MT, 0, P.stream>>>(A);
    }
    HIP_TRY(hipGetLastError());
}

void run_leaf_solve(Pipeline &P, void *z)
{
    const Plan &p = *P.plan;
    LeafArgs A = leaf_args(P);
    if (p.leafmax > LEAF_LDS_MAX) {
        ProfScope ps(P.stream, PS_LEAF_SOLVE);
        if (p.f32())
            leaf_solve_big_kernel<float><<<(unsigned)p.nleaf, LEAF_MT, 0, P.stream>>>(A, (float *)z);
        else
            leaf_solve_big_kernel<double><<<(unsigned)p.nleaf, LEAF_MT, 0, P.stream>>>(A, (double *)z);
        HIP_TRY(hipGetLastError());
        return;
    }
    static bool attr = false;   // room for the packed factor of a 128-point leaf (66 KB)
    if (!attr) {
        const int most = sizeof(double) * LEAF_LDS_MAX * (LEAF_LDS_MAX + 1) / 2;
        HIP_TRY(hipFuncSetAttribute((const void *)leaf_solve_kernel<float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, most));
        HIP_TRY(hipFuncSetAttribute((const void *)leaf_solve_kernel<double>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, most));
        attr = true;
    }
    const size_t lds = sizeof(double) * (size_t)p.leafmax * (p.leafmax + 1) / 2;
    ProfScope ps(P.stream, PS_LEAF_SOLVE);
    if (p.f32())
        leaf_solve_kernel<float><<<(unsigned)p.nleaf, LEAF_SOLVE_T, lds, P.stream>>>(A, (float *)z);
    else
        leaf_solve_kernel<double><<<(unsigned)p.nleaf, LEAF_SOLVE_T, lds, P.stream>>>(A, (double *)z);
    HIP_TRY(hipGetLastError());
}

}  // namespace hodlr
