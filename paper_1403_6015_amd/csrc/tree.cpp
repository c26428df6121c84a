// Host side of the tree: point ordering, node ranges, column layout of the
// basis panels and the launch tables of the device stages.
//
// Ordering (§3 of the paper: points are sorted by a k-d tree, one dimension at
// a time, and the resulting order makes matrix rows/columns correspond to
// tree nodes).  The tree is count-based: a node of m consecutive points splits
// into a left child of floor(m/2) points and a right child of the rest.  The
// number of levels is the smallest L with every leaf holding at most `leaf`
// points (the paper's kappa from the smallest block size p_max, §3.2).
#include <algorithm>
#include <cstring>
#include <numeric>

#include "common.h"

namespace hodlr {

int num_levels(int64_t n, int leaf)
{
    if (n < 1 || leaf < 1)
        return 0;
    int L = 0;
    while (L < 62 && (n + ((int64_t)1 << L) - 1) / ((int64_t)1 << L) > leaf)
        ++L;
    return L;
}

void order_points(const double *x, int64_t n, int dim, int leaf, int64_t *perm)
{
    std::vector<int64_t> p(n);
    std::iota(p.begin(), p.end(), 0);
    auto by = [&](int c) {
        return [&, c](int64_t a, int64_t b) {
            double xa = x[a * dim + c], xb = x[b * dim + c];
            return xa < xb || (xa == xb && a < b);
        };
    };
    if (dim == 1) {
        std::sort(p.begin(), p.end(), by(0));
    } else {
        int L = num_levels(n, leaf);
        // depth-d nodes: recursive halving of [0, n)
        std::vector<std::pair<int64_t, int64_t>> level{{0, n}};
        for (int d = 0; d < L; ++d) {
            int c = d % dim;
            std::vector<std::pair<int64_t, int64_t>> next;
            next.reserve(level.size() * 2);
            for (auto [s, e] : level) {
                std::sort(p.begin() + s, p.begin() + e, by(c));
                int64_t m = s + (e - s) / 2;
                next.push_back({s, m});
                next.push_back({m, e});
            }
            level.swap(next);
        }
    }
    std::memcpy(perm, p.data(), sizeof(int64_t) * (size_t)n);
}

static void make_chunks(int node, int side, int64_t lo, int64_t hi, int64_t size,
                        std::vector<Chunk> &out, int &slot)
{
    for (int64_t a = lo; a < hi; a += size) {
        Chunk c;
        c.node = node;
        c.side = side;
        c.lo = a;
        c.hi = std::min(hi, a + size);
        c.part = slot++;
        c.pad_ = 0;
        out.push_back(c);
    }
}

void plan_build(Plan &p, int64_t n, int dim, int leaf, const hodlr_opts *opts, int lvl_rows,
                int red_cols, int red_grp)
{
    if (red_grp != 8 && red_grp != 64)
        throw Error{HODLR_EINVAL, "reduce_group must be 8 or 64"};
    p.red_grp = red_grp;
    if (lvl_rows != 256 && lvl_rows != 512 && lvl_rows != 1024)
        throw Error{HODLR_EINVAL, "level_rows must be 256, 512 or 1024"};
    if (red_cols != 4 && red_cols != 8)
        throw Error{HODLR_EINVAL, "reduce_cols must be 4 or 8"};
    p.lvl_rows = lvl_rows;
    p.red_cols = red_cols;
    p.n = n;
    p.dim = dim;
    p.leaf = leaf;
    p.L = num_levels(n, leaf);
    p.cap = opts ? opts->max_rank : 64;
    p.precision = opts ? opts->precision : HODLR_FP64;
    p.refine_tol = (opts && opts->refine_tol > 0) ? opts->refine_tol : 1e-10;
    p.max_refine = opts ? opts->max_refine : 8;   // checked >= 0 by the entry points
    p.refine = p.precision == HODLR_MIXED || (opts && opts->refine);
    p.mixed_check = p.precision == HODLR_MIXED && !(opts && opts->mixed_unchecked);
    p.compressor = opts ? opts->compressor : HODLR_COMPRESS_ACA;
    p.level_form = opts ? opts->level_form : 0;
    const int L = p.L;
    const int64_t nn = ((int64_t)2 << L) - 1;
    p.nint = ((int64_t)1 << L) - 1;
    p.nleaf = (int64_t)1 << L;
    p.start.assign(nn, 0);
    p.end.assign(nn, 0);
    p.start[0] = 0;
    p.end[0] = n;
    for (int64_t h = 0; h < p.nint; ++h) {
        int64_t s = p.start[h], e = p.end[h], m = s + (e - s) / 2;
        p.start[2 * h + 1] = s;
        p.end[2 * h + 1] = m;
        p.start[2 * h + 2] = m;
        p.end[2 * h + 2] = e;
    }
    p.leafmax = 0;
    for (int64_t h = p.nint; h < nn; ++h)
        p.leafmax = std::max<int>(p.leafmax, (int)(p.end[h] - p.start[h]));

    // columns reserved per depth j (bases of depth-j nodes, rank of the parent block)
    p.capj.assign(L + 2, 0);
    p.cofa.assign(L + 2, 0);
    for (int j = 1; j <= L; ++j) {
        int64_t best = 0;
        for (int64_t h = p.first_at(j - 1); h < p.first_at(j); ++h) {
            int64_t s = p.start[h], e = p.end[h], m = s + (e - s) / 2;
            best = std::max(best, std::min(m - s, e - m));
        }
        p.capj[j] = (int)std::min<int64_t>(p.cap, best);
    }
    p.cofa[1] = 1;
    for (int j = 1; j <= L; ++j)
        p.cofa[j + 1] = p.cofa[j] + p.capj[j];
    p.ncol = (L >= 1) ? p.cofa[L + 1] : 1;

    // cross-approximation tables: blocks whose sides fit ACA_SMALL run whole in
    // one work-group; larger ones get per-pass chunks (row passes sweep beta,
    // column passes sweep alpha), longer ones for 1-D points (low ranks)
    p.aca_chunk = dim == 1 ? ACA_CHUNK_1D : ACA_CHUNK_ND;
    p.aca_small.clear();
    p.aca_big.clear();
    p.aca_row.clear();
    p.aca_col.clear();
    p.aca_rowidx.clear();
    p.aca_colidx.clear();
    p.aca_nrow.clear();
    p.aca_ncol.clear();
    p.aca_rowbase.clear();
    p.aca_colbase.clear();
    p.pad_chunks.clear();
    p.aca_big_active = 0;
    int rslot = 0, cslot = 0, pslot = 0;
    std::vector<int> tiny;   // small blocks with both sides <= ACA_TINY, listed last
    for (int64_t h = 0; h < p.nint; ++h) {
        int64_t s = p.start[h], e = p.end[h], m = s + (e - s) / 2;
        if (m - s == 0 || e - m == 0 || p.cap == 0)
            continue;
        make_chunks((int)h, 0, s, m, 4096, p.pad_chunks, pslot);
        make_chunks((int)h, 1, m, e, 4096, p.pad_chunks, pslot);
        if (m - s <= ACA_SMALL && e - m <= ACA_SMALL) {
            if (m - s <= ACA_TINY && e - m <= ACA_TINY)
                tiny.push_back((int)h);
            else
                p.aca_small.push_back((int)h);
            continue;
        }
        int b = (int)p.aca_big.size();
        p.aca_big.push_back((int)h);
        p.aca_big_active += 1;
        p.aca_rowbase.push_back(rslot);
        p.aca_colbase.push_back(cslot);
        make_chunks((int)h, 1, m, e, p.aca_chunk, p.aca_row, rslot);
        make_chunks((int)h, 0, s, m, p.aca_chunk, p.aca_col, cslot);
        p.aca_nrow.push_back(rslot - p.aca_rowbase.back());
        p.aca_ncol.push_back(cslot - p.aca_colbase.back());
        while ((int)p.aca_rowidx.size() < rslot)
            p.aca_rowidx.push_back(b);
        while ((int)p.aca_colidx.size() < cslot)
            p.aca_colidx.push_back(b);
    }
    p.aca_small_wide = (int)p.aca_small.size();
    p.aca_small.insert(p.aca_small.end(), tiny.begin(), tiny.end());
    p.aca_pw = std::max(p.cap, 1) + 4;

    // level tables: for depth d, chunks over the rows of each child of each node
    p.lvl.assign(L, {});
    p.lvl_nch.assign(L, {});
    p.lvl_base.assign(L, {});
    for (int d = 0; d < L; ++d) {
        int slot = 0;
        for (int64_t h = p.first_at(d); h < p.first_at(d + 1); ++h) {
            p.lvl_base[d].push_back(slot);
            int64_t s = p.start[h], e = p.end[h], m = s + (e - s) / 2;
            for (int side = 0; side < 2; ++side) {
                int64_t lo = side ? m : s, hi = side ? e : m;
                int64_t len = hi - lo;
                const int64_t csz = p.lvl_rows;   // the small-rank kernels assume this
                if (len > 0)
                    make_chunks((int)h, side, lo, hi, csz, p.lvl[d], slot);
            }
            p.lvl_nch[d].push_back(slot - p.lvl_base[d].back());
        }
    }
    p.lvl_maxlen.assign(L, 0);
    for (int d = 0; d < L; ++d)
        for (const Chunk &c : p.lvl[d])
            p.lvl_maxlen[d] = std::max(p.lvl_maxlen[d], (int)(c.hi - c.lo));
    // sketch compressor tables
    p.sk.assign(p.compressor == HODLR_COMPRESS_SKETCH ? L : 0, {});
    p.sk_abase.assign(p.sk.size(), {});
    p.sk_acnt.assign(p.sk.size(), {});
    for (int d = 0; d < (int)p.sk.size(); ++d) {
        int aslot = 0;
        for (int64_t h = p.first_at(d); h < p.first_at(d + 1); ++h) {
            int64_t s = p.start[h], e = p.end[h], m = s + (e - s) / 2;
            p.sk_abase[d].push_back(aslot);
            int bslot = 0;
            make_chunks((int)h, 0, s, m, SK_ROWS, p.sk[d], aslot);
            p.sk_acnt[d].push_back(aslot - p.sk_abase[d].back());
            const size_t b0 = p.sk[d].size();
            make_chunks((int)h, 1, m, e, SK_ROWS, p.sk[d], bslot);
            for (size_t c = b0; c < p.sk[d].size(); ++c)
                p.sk[d][c].part = -1;
        }
    }
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Host image of the plan's device tables; offsets are kept in the plan so
// the same image can be bound to any device region (plan_bind).
size_t plan_image(Plan &p, std::vector<char> &host)
{
    const int L = p.L;
    const int64_t nn = ((int64_t)2 << L) - 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    auto &o = p.tbl;
    o.start = take(sizeof(int64_t) * nn);
    o.end = take(sizeof(int64_t) * nn);
    o.ar = take(sizeof(Chunk) * std::max<size_t>(1, p.aca_row.size()));
    o.ac = take(sizeof(Chunk) * std::max<size_t>(1, p.aca_col.size()));
    o.pc = take(sizeof(Chunk) * std::max<size_t>(1, p.pad_chunks.size()));
    const size_t nbig = std::max<size_t>(1, p.aca_big.size());
    o.nr = take(sizeof(int) * nbig);
    o.nc = take(sizeof(int) * nbig);
    o.rb = take(sizeof(int) * nbig);
    o.cb = take(sizeof(int) * nbig);
    o.bg = take(sizeof(int) * nbig);
    o.sm = take(sizeof(int) * std::max<size_t>(1, p.aca_small.size()));
    o.ri = take(sizeof(int) * std::max<size_t>(1, p.aca_rowidx.size()));
    o.ci = take(sizeof(int) * std::max<size_t>(1, p.aca_colidx.size()));
    o.l.assign(L, 0);
    o.ln.assign(L, 0);
    o.lb.assign(L, 0);
    for (int d = 0; d < L; ++d) {
        o.l[d] = take(sizeof(Chunk) * std::max<size_t>(1, p.lvl[d].size()));
        o.ln[d] = take(sizeof(int) * p.lvl_nch[d].size());
        o.lb[d] = take(sizeof(int) * p.lvl_base[d].size());
    }
    const int LK = (int)p.sk.size();
    o.k.assign(LK, 0);
    o.ka.assign(LK, 0);
    o.kc.assign(LK, 0);
    for (int d = 0; d < LK; ++d) {
        o.k[d] = take(sizeof(Chunk) * std::max<size_t>(1, p.sk[d].size()));
        o.ka[d] = take(sizeof(int) * p.sk_abase[d].size());
        o.kc[d] = take(sizeof(int) * p.sk_acnt[d].size());
    }
    host.assign(off, 0);
    auto put = [&](size_t at, const void *src, size_t bytes) {
        if (bytes)
            std::memcpy(host.data() + at, src, bytes);
    };
    put(o.start, p.start.data(), sizeof(int64_t) * nn);
    put(o.end, p.end.data(), sizeof(int64_t) * nn);
    put(o.ar, p.aca_row.data(), sizeof(Chunk) * p.aca_row.size());
    put(o.ac, p.aca_col.data(), sizeof(Chunk) * p.aca_col.size());
    put(o.pc, p.pad_chunks.data(), sizeof(Chunk) * p.pad_chunks.size());
    put(o.nr, p.aca_nrow.data(), sizeof(int) * p.aca_nrow.size());
    put(o.nc, p.aca_ncol.data(), sizeof(int) * p.aca_ncol.size());
    put(o.rb, p.aca_rowbase.data(), sizeof(int) * p.aca_rowbase.size());
    put(o.cb, p.aca_colbase.data(), sizeof(int) * p.aca_colbase.size());
    put(o.bg, p.aca_big.data(), sizeof(int) * p.aca_big.size());
    put(o.sm, p.aca_small.data(), sizeof(int) * p.aca_small.size());
    put(o.ri, p.aca_rowidx.data(), sizeof(int) * p.aca_rowidx.size());
    put(o.ci, p.aca_colidx.data(), sizeof(int) * p.aca_colidx.size());
    for (int d = 0; d < L; ++d) {
        put(o.l[d], p.lvl[d].data(), sizeof(Chunk) * p.lvl[d].size());
        put(o.ln[d], p.lvl_nch[d].data(), sizeof(int) * p.lvl_nch[d].size());
        put(o.lb[d], p.lvl_base[d].data(), sizeof(int) * p.lvl_base[d].size());
    }
    for (int d = 0; d < LK; ++d) {
        put(o.k[d], p.sk[d].data(), sizeof(Chunk) * p.sk[d].size());
        put(o.ka[d], p.sk_abase[d].data(), sizeof(int) * p.sk_abase[d].size());
        put(o.kc[d], p.sk_acnt[d].data(), sizeof(int) * p.sk_acnt[d].size());
    }
    return off;
}

void plan_bind(Plan &p, char *b)
{
    const auto &o = p.tbl;
    p.d_start = (int64_t *)(b + o.start);
    p.d_end = (int64_t *)(b + o.end);
    p.d_aca_row = (Chunk *)(b + o.ar);
    p.d_aca_col = (Chunk *)(b + o.ac);
    p.d_pad_chunks = (Chunk *)(b + o.pc);
    p.d_aca_nrow = (int *)(b + o.nr);
    p.d_aca_ncol = (int *)(b + o.nc);
    p.d_aca_rowbase = (int *)(b + o.rb);
    p.d_aca_colbase = (int *)(b + o.cb);
    p.d_aca_big = (int *)(b + o.bg);
    p.d_aca_small = (int *)(b + o.sm);
    p.d_aca_rowidx = (int *)(b + o.ri);
    p.d_aca_colidx = (int *)(b + o.ci);
    p.d_lvl.resize(p.L);
    p.d_lvl_nch.resize(p.L);
    p.d_lvl_base.resize(p.L);
    for (int d = 0; d < p.L; ++d) {
        p.d_lvl[d] = (Chunk *)(b + o.l[d]);
        p.d_lvl_nch[d] = (int *)(b + o.ln[d]);
        p.d_lvl_base[d] = (int *)(b + o.lb[d]);
    }
    const int LK = (int)p.sk.size();
    p.d_sk.resize(LK);
    p.d_sk_abase.resize(LK);
    p.d_sk_acnt.resize(LK);
    for (int d = 0; d < LK; ++d) {
        p.d_sk[d] = (Chunk *)(b + o.k[d]);
        p.d_sk_abase[d] = (int *)(b + o.ka[d]);
        p.d_sk_acnt[d] = (int *)(b + o.kc[d]);
    }
}

void plan_upload(Plan &p)
{
    HIP_TRY(hipGetDevice(&p.device));
    std::vector<char> host;
    size_t off = plan_image(p, host);
    void *dev = nullptr;
    if (hipMalloc(&dev, std::max<size_t>(off, 256)) != hipSuccess)
        throw Error{HODLR_ENOMEM, "device allocation of plan tables failed"};
    if (hipMemcpy(dev, host.data(), off, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dev);
        throw Error{HODLR_EDEVICE, "upload of plan tables failed"};
    }
    p.dev_tables = dev;
    p.dev_tables_bytes = off;
    plan_bind(p, (char *)dev);
}

void plan_release(Plan &p)
{
    if (p.dev_tables) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p.device);
        (void)hipFree(p.dev_tables);
        (void)hipSetDevice(cur);
    }
    p.dev_tables = nullptr;
}

Layout make_layout(const Plan &p, bool store_leaf)
{
    Layout y{};
    const int L = p.L;
    const int64_t n = p.n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 8));
        return o;
    };
    int capmax = 1;
    for (int j = 1; j <= L; ++j)
        capmax = std::max(capmax, p.capj[j]);
    y.store_leaf = store_leaf;
    y.W = take(sizeof(double) * (size_t)n * (size_t)p.ncol);
    y.Xt = take(p.panel_bytes() * (size_t)n * (size_t)p.ncol);
    int64_t lm = p.leafmax;
    y.G = take(store_leaf ? sizeof(double) * (size_t)p.nleaf * (size_t)(lm * (lm + 1) / 2) : 8);
    // leaves above LEAF_LDS_MAX: 8 x 8 tiles of 16 x 16 doubles each for L21
    y.L21 = take(lm > LEAF_LDS_MAX ? sizeof(double) * (size_t)p.nleaf * 64 * 256 : 8);
    int64_t ni = std::max<int64_t>(p.nint, 1);
    int64_t nb = std::max<int64_t>((int64_t)p.aca_big.size(), 1);
    y.aca_state = take(sizeof(BigState) * 2 * nb);
    y.aca_used = take(sizeof(int) * nb * USED_MAX);
    y.aca_vdots = take(sizeof(double) * nb * RMAX_ABS);
    y.aca_part = take(sizeof(double) * (p.aca_row.size() + p.aca_col.size()) * p.aca_pw);
    y.aca_status = take(sizeof(int) * ni);
    y.rank = take(sizeof(int) * ni);
    y.leaf_ld = take(sizeof(double) * p.nleaf);
    y.node_ld = take(sizeof(double) * ni);
    // worst-case sizes from the reserved columns
    int64_t lp = 1, tb = 1;
    for (int d = 0; d < L; ++d) {
        int64_t cntc = p.cofa[d + 2];           // columns 0 .. end of panel d+1
        int64_t r = p.capj[d + 1];
        lp = std::max<int64_t>(lp, (int64_t)p.lvl[d].size() * r * cntc);
        // records of level d-1 written by level d's fused update
        if (d > 0)
            lp = std::max<int64_t>(lp, (int64_t)p.lvl[d].size() * p.capj[d] * p.cofa[d + 1]);
        tb = std::max<int64_t>(tb, (p.first_at(d + 1) - p.first_at(d)) * 2 * r * cntc);
    }
    y.lvl_part_cap = lp;
    y.lvl_part = take(sizeof(double) * lp);
    y.Tbuf = take(sizeof(double) * tb);
    y.Sbuf = take(sizeof(double) * tb);
    // per node: LU of I - QP, P, Q and pivots; above RMAX_LDS also N^{-1}
    y.small_stride = (capmax > RMAX_LDS ? 4 : 3) * (int64_t)capmax * capmax + capmax;
    y.small = take(sizeof(double) * ni * y.small_stride);
    y.dot_part = take(sizeof(double) * 1024);
    y.out = take(sizeof(double) * 8);
    y.status = take(sizeof(int) * 4);
    y.cols = take(sizeof(int) * p.ncol);
    y.misc = take(4096);
    // sketch compressor: one level's sketches (n rows), its partial cores (one
    // per alpha chunk), its cores and its factor maps (one per node)
    size_t skp = 1, skn = 1;
    for (int d = 0; d < (int)p.sk.size(); ++d) {
        size_t na = 0;
        for (int c : p.sk_acnt[d])
            na += (size_t)c;
        skp = std::max(skp, na);
        skn = std::max<size_t>(skn, (size_t)(p.first_at(d + 1) - p.first_at(d)));
    }
    const bool sk = !p.sk.empty();
    y.sk_buf = take(sk ? sizeof(double) * (size_t)n * SK_SPMAX : 8);
    y.sk_part = take(sk ? sizeof(double) * skp * SK_SPMAX * SK_SMAX : 8);
    y.sk_core = take(sk ? sizeof(double) * skn * SK_SPMAX * SK_SMAX : 8);
    y.sk_fac = take(sk ? sizeof(double) * skn * (SK_SMAX + SK_SPMAX) * SK_CAP_MAX : 8);
    y.total = off;
    return y;
}

}  // namespace hodlr
