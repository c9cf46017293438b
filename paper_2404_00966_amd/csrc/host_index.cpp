// Index construction and streamed updates (host orchestration; the distance
// work runs in GPU kernels).
//
// Construction follows Sec. 4.3 with global pivots.  m pivots are chosen once
// by farthest-first traversal (the FFT rule of Algorithm 2, first pivot
// seeded) and every object's distance to every one of them is kept in a
// pivot table.  The tree has the paper's shape (fanout F, equal-count leaves
// from the leaf size or the height rule of Sec. 4.2), but the order of the
// objects comes from K farthest-first centres run on the GPU: every object
// joins the cell of its nearest centre, cells follow a nearest-neighbour
// chain of their centres, objects inside a cell follow their distance to the
// centre, and each equal-count leaf boundary moves to a cell boundary within
// half a leaf.  A node covers its F children's runs.  Every node keeps the box
// [min, max] of its objects' distances to every global pivot, which is what
// the query-time filters test (Lemma 1 on all pivots at once); every leaf
// keeps a pivot of its own and its covering radius.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>

#include "gts_internal.h"
#include "kernels.h"

namespace gts {

namespace {

uint64_t splitmix64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int pad_pivots(int m) { return m <= 8 ? 8 : (m <= 16 ? 16 : 32); }

// Stage timer for the build, printed to stderr when GTS_VERBOSE is set.
struct StageClock {
    bool on = std::getenv("GTS_VERBOSE") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void mark(const char *what) {
        if (!on) return;
        auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[gts build] %-28s %8.1f ms\n", what,
                     std::chrono::duration<double, std::milli>(now - t).count());
        t = now;
    }
};

// Number of partition layers: the paper's height rule, or the smallest depth
// whose average leaf holds at most leaf_size objects.
int choose_levels(int64_t n, int F, int leaf_size)
{
    if (leaf_size > 0) {
        int L = 0;
        long double cap = 1.0L;
        while ((long double)n / cap > (long double)leaf_size && L < 30) {
            cap *= F;
            L++;
        }
        return L;
    }
    int e = 0;
    long double p = 1.0L;
    while (p < (long double)(n + 1)) {
        p *= F;
        e++;
    }
    return std::max(0, e - 2);
}

// Blocking upload: the sources are often temporaries of the caller.
template <class T> void upload(DevBuf &b, const std::vector<T> &v, hipStream_t st)
{
    b.alloc(std::max<size_t>(v.size() * sizeof(T), 16));
    if (!v.empty()) {
        GTS_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        GTS_HIP(hipStreamSynchronize(st));
    }
}

}  // namespace

void rows_to_device(float *dst, int dp, const float *src, int dim, int64_t n, bool src_on_device, hipStream_t st)
{
    if (n == 0) return;
    if (src_on_device) {
        // (a fill kernel rather than a memset: this copy may be recorded
        // into a graph)
        if (dp != dim) k::fill_u32(reinterpret_cast<uint32_t *>(dst), (int64_t)n * dp, 0u, st);
        GTS_HIP(hipMemcpy2DAsync(dst, dp * sizeof(float), src, dim * sizeof(float), dim * sizeof(float), n,
                                 hipMemcpyDeviceToDevice, st));
    } else if (dp == dim) {
        GTS_HIP(hipMemcpyAsync(dst, src, (size_t)n * dim * sizeof(float), hipMemcpyHostToDevice, st));
        GTS_HIP(hipStreamSynchronize(st));
    } else {
        std::vector<float> packed((size_t)n * dp, 0.f);
        for (int64_t i = 0; i < n; i++)
            std::copy(src + (size_t)i * dim, src + (size_t)(i + 1) * dim, &packed[(size_t)i * dp]);
        GTS_HIP(hipMemcpyAsync(dst, packed.data(), packed.size() * sizeof(float), hipMemcpyHostToDevice, st));
        GTS_HIP(hipStreamSynchronize(st));
    }
}

void alphabet_add(gts_index *idx, const std::vector<uint8_t> &chars)
{
    bool seen[256] = {};
    for (uint8_t b : chars) seen[b] = true;
    bool grew = !idx->lut.p;
    for (int b = 0; b < 256; b++)
        if (seen[b] && !idx->alpha[b]) {
            idx->alpha[b] = true;
            grew = true;
        }
    if (!grew) return;
    std::vector<uint8_t> lut(256);
    int code = 0;
    for (int b = 0; b < 256; b++)
        if (idx->alpha[b]) lut[b] = (uint8_t)code++;
    for (int b = 0; b < 256; b++)
        if (!idx->alpha[b]) lut[b] = (uint8_t)code;   // the all-zero row
    idx->arows = code + 1;
    upload(idx->lut, lut, idx->stream);
}

namespace {

// Tree shape: levels, node ids of the leaves, node count (Eq. 1 numbering).
void tree_shape(gts_index *idx, int64_t n)
{
    Tree &t = idx->data.tree;
    const int F = idx->fanout;
    t.mpad = pad_pivots(idx->num_pivots);
    t.fanout = F;
    t.levels = choose_levels(n, F, idx->opts.leaf_size);
    {
        long double nn = 0, lv = 1;
        for (int l = 0; l <= t.levels; l++) {
            nn += lv;
            lv *= F;
        }
        GTS_CHECK(nn < (long double)(1 << 26), GTS_ENOTSUP, "tree too deep for this fanout (more than 2^26 nodes)");
    }
    t.n_nodes = 1;
    t.n_leaves = 1;
    t.leaf0 = 0;
    for (int l = 0; l < t.levels; l++) {
        t.leaf0 = t.leaf0 * F + 1;
        t.n_leaves *= F;
        t.n_nodes += t.n_leaves;
    }
}

// Nearest-neighbour chain over K centres from their distance matrix dk
// [K][K]: rank[c] = place of centre c on the chain (centre 0 first).
void centre_chain(const std::vector<float> &dk, int K, std::vector<int32_t> &rank, std::vector<int32_t> &by_rank)
{
    rank.assign(K, -1);
    by_rank.assign(K, 0);
    int at = 0;
    rank[0] = 0;
    for (int r = 1; r < K; r++) {
        int best = -1;
        for (int c = 0; c < K; c++)
            if (rank[c] < 0 && (best < 0 || dk[(size_t)at * K + c] < dk[(size_t)at * K + best])) best = c;
        rank[best] = r;
        by_rank[r] = best;
        at = best;
    }
}

// Leaf cuts: equal-count boundaries, each moved to the nearest cell boundary
// (a position whose cell differs from the previous one's) within half a
// leaf.  bnd ascending; cut[L] = n.
std::vector<int64_t> leaf_cuts(const std::vector<int64_t> &bnd, int64_t n, int64_t L)
{
    std::vector<int64_t> cut(L + 1, 0);
    cut[L] = n;
    for (int64_t i = 1; i < L; i++) {
        const int64_t ideal = (int64_t)((long double)i * n / L);
        int64_t c = std::max(ideal, cut[i - 1]);
        auto it = std::lower_bound(bnd.begin(), bnd.end(), ideal);
        int64_t best = -1;
        if (it != bnd.end()) best = *it;
        if (it != bnd.begin() && (best < 0 || ideal - *(it - 1) < best - ideal)) best = *(it - 1);
        if (best >= 0 && 2 * std::llabs(best - ideal) * L <= n && best > cut[i - 1]) c = best;
        cut[i] = std::min(c, n);
    }
    return cut;
}

// ---------------------------------------------------------------------------
// L2: every n-sized step on the device.  Global pivots by farthest-first
// traversal over all objects (the FFT rule, first pivot seeded) and the
// pivot table from their rows; K farthest-first centres over a strided
// sample of the objects, every object into the cell of its nearest centre
// (bf16 MFMA search; the cells only order the objects), cells along the
// nearest-neighbour chain of their centres and objects inside a cell by
// distance to the centre (a stable device radix sort); the leaf cuts on the
// host from the cell of each position; then the object table, pivot table,
// node boxes, slab summaries and leaf pivots formed in leaf order in HBM.
// perm[p] = input row of position p.
// ---------------------------------------------------------------------------
void build_l2(gts_index *idx, const HostObjects &objs, DevBuf *rows, StageClock &clock, std::vector<int32_t> &perm)
{
    hipStream_t st = idx->stream;
    IndexData &d = idx->data;
    Tree &t = d.tree;
    const int64_t n = objs.count();
    const int m = d.m, mpad = t.mpad;
    d.dim = objs.dim;
    d.dp = (objs.dim + 3) / 4 * 4;
    d.ksteps = (objs.dim + 31) / 32;
    const int dp = d.dp;
    const bool l1 = idx->l1;                 // Manhattan: no bf16 tables at all
    const bool mfma = d.dim <= kMaxMfmaDim && !l1;
    // the rows in input order, on the device (given, or uploaded from the host)
    DevBuf in_x;
    if (rows) {
        in_x = std::move(*rows);
        GTS_CHECK(in_x.bytes >= (size_t)n * dp * sizeof(float), GTS_EINVAL, "build: device rows too short");
    } else {
        in_x.alloc((size_t)n * dp * sizeof(float));
        rows_to_device(in_x.as<float>(), dp, objs.vecs.data(), objs.dim, n, false, st);
    }
    clock.mark("upload");

    // ---- global pivots and the pivot table (input order) --------------------
    uint64_t rng = idx->opts.seed ? idx->opts.seed : 0x2404009660ULL;
    const int64_t first = (int64_t)(splitmix64(&rng) % (uint64_t)n);
    DevBuf keys, dcent, mind, nearc;
    {
        std::vector<uint64_t> hk((size_t)m + 1, 0ull);
        hk[0] = (uint64_t)(0xffffffffu - (uint32_t)first);
        upload(keys, hk, st);
    }
    dcent.alloc((size_t)std::max(m, 1) * sizeof(int32_t));
    mind.alloc((size_t)n * sizeof(float));
    nearc.alloc((size_t)n * sizeof(int32_t));
    k::fft_centers_l2(in_x.as<float>(), n, dp, m, keys.as<uint64_t>(), dcent.as<int32_t>(), mind.as<float>(),
                      nearc.as<int32_t>(), st, l1);
    d.P32.alloc((size_t)std::max(m, 1) * dp * sizeof(float));
    k::gather_rows(in_x.as<float>(), dp, dcent.as<int32_t>(), m, d.P32.as<float>(), st);
    DevBuf pt_in;
    pt_in.alloc((size_t)mpad * n * sizeof(float));
    k::dist_l2_pivots(in_x.as<float>(), n, d.P32.as<float>(), m, mpad, dp, pt_in.as<float>(), n, 1, st, l1);
    clock.mark("global pivots + table");

    // ---- cells: farthest-first centres, nearest centre of every object -----
    const int K = (int)std::max<int64_t>(1, std::min<int64_t>({t.n_leaves / 8, (int64_t)kMaxCentres, n}));
    // the centres come from a strided sample unless the rows are too wide for
    // either nearest-centre search (then the traversal runs over every object
    // and gives each its nearest centre itself)
    const bool sampled = mfma || (int64_t)dp * sizeof(float) <= ((int64_t)48 << 10);
    const int64_t S = sampled ? std::min<int64_t>(n, std::max<int64_t>(16384, 32 * (int64_t)K)) : n;
    DevBuf sx, dsidx;
    std::vector<int32_t> sidx;
    const float *fx = in_x.as<float>();
    if (S < n) {
        sidx.resize(S);
        for (int64_t s = 0; s < S; s++) sidx[s] = (int32_t)((long double)s * n / S);
        upload(dsidx, sidx, st);
        sx.alloc((size_t)S * dp * sizeof(float));
        k::gather_rows(in_x.as<float>(), dp, dsidx.as<int32_t>(), S, sx.as<float>(), st);
        fx = sx.as<float>();
    }
    uint64_t crng = (idx->opts.seed ? idx->opts.seed : 0x2404009660ULL) ^ 0x5bd1e9955bd1e995ULL;
    const int64_t first_centre = (int64_t)(splitmix64(&crng) % (uint64_t)S);
    DevBuf ckeys, ccent, cmind, cnear;
    {
        std::vector<uint64_t> hk((size_t)K + 1, 0ull);
        hk[0] = (uint64_t)(0xffffffffu - (uint32_t)first_centre);
        upload(ckeys, hk, st);
    }
    ccent.alloc((size_t)K * sizeof(int32_t));
    cmind.alloc((size_t)S * sizeof(float));
    cnear.alloc((size_t)S * sizeof(int32_t));
    k::fft_centers_l2(fx, S, dp, K, ckeys.as<uint64_t>(), ccent.as<int32_t>(), cmind.as<float>(),
                      cnear.as<int32_t>(), st, l1);
    std::vector<int32_t> cent(K);
    GTS_HIP(hipMemcpyAsync(cent.data(), ccent.p, (size_t)K * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GTS_HIP(hipStreamSynchronize(st));
    if (S < n)
        for (int c = 0; c < K; c++) cent[c] = sidx[cent[c]];
    DevBuf dcentres, cx;
    upload(dcentres, cent, st);
    const int64_t Kp = (K + 63) / 64 * 64;
    cx.alloc((size_t)Kp * dp * sizeof(float));
    GTS_HIP(hipMemsetAsync(cx.p, 0, (size_t)Kp * dp * sizeof(float), st));
    k::gather_rows(in_x.as<float>(), dp, dcentres.as<int32_t>(), K, cx.as<float>(), st);
    const int32_t *cell = cnear.as<int32_t>();
    int cstride = 1;
    DevBuf c16, cn, ce, x16, xn_in, xe_in, near8;
    if (S < n && !mfma) {
        // exact float32 nearest centre (Manhattan, or rows wider than 128)
        near8.alloc((size_t)n * sizeof(int32_t));
        k::nearest_centre(in_x.as<float>(), dp, n, cx.as<float>(), K, l1, near8.as<int32_t>(), st);
        cell = near8.as<int32_t>();
    } else if (S < n) {
        // nearest centre by bf16 MFMA estimates (padding centres never win)
        c16.alloc((size_t)Kp * d.ksteps * 32 * sizeof(uint16_t));
        cn.alloc((size_t)Kp * sizeof(float));
        ce.alloc((size_t)Kp * sizeof(float));
        k::rows_bf16(cx.as<float>(), K, Kp, d.dim, dp, d.ksteps, c16.as<uint16_t>(), cn.as<float>(), ce.as<float>(),
                     INFINITY, st);
        const int64_t n16 = (n + 15) / 16 * 16;
        x16.alloc((size_t)n16 * d.ksteps * 32 * sizeof(uint16_t));
        xn_in.alloc((size_t)n16 * sizeof(float));
        xe_in.alloc((size_t)n16 * sizeof(float));
        k::rows_bf16(in_x.as<float>(), n, n16, d.dim, dp, d.ksteps, x16.as<uint16_t>(), xn_in.as<float>(),
                     xe_in.as<float>(), 0.f, st);
        near8.alloc((size_t)n16 * k::kNearLeaves * sizeof(int32_t));
        k::leaf_near(c16.as<uint16_t>(), cn.as<float>(), Kp, d.ksteps, x16.as<uint16_t>(), n, near8.as<int32_t>(), st);
        cell = near8.as<int32_t>();
        cstride = k::kNearLeaves;
    }
    DevBuf cdist;
    cdist.alloc((size_t)n * sizeof(float));
    k::centre_dist(in_x.as<float>(), dp, n, cell, cstride, cx.as<float>(), cdist.as<float>(), st, l1);
    clock.mark("centres");
    // centre-to-centre distances, then the chain (host, K x K)
    std::vector<float> dk((size_t)K * K);
    {
        DevBuf ddk;
        ddk.alloc(dk.size() * sizeof(float));
        k::dist_l2_pivots(cx.as<float>(), K, cx.as<float>(), K, K, dp, ddk.as<float>(), K, 1, st, l1);
        GTS_HIP(hipMemcpyAsync(dk.data(), ddk.p, dk.size() * sizeof(float), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipStreamSynchronize(st));
    }
    std::vector<int32_t> rank, by_rank;
    centre_chain(dk, K, rank, by_rank);
    // the leaf order: (cell rank, distance to the centre, input row)
    DevBuf drank, okey, operm, stmp;
    upload(drank, rank, st);
    okey.alloc((size_t)n * sizeof(uint32_t));
    operm.alloc((size_t)n * sizeof(int32_t));
    const size_t sb = k::sort_pairs_bytes(n);
    stmp.alloc(sb);
    k::cell_order(cdist.as<float>(), cell, cstride, drank.as<int32_t>(), K, n, okey.as<uint32_t>(),
                  operm.as<int32_t>(), stmp.p, sb, st);
    std::vector<uint32_t> prank(n);
    perm.resize(n);
    GTS_HIP(hipMemcpyAsync(prank.data(), okey.p, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GTS_HIP(hipMemcpyAsync(perm.data(), operm.p, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GTS_HIP(hipStreamSynchronize(st));
    std::vector<int64_t> bnd;   // positions where a new cell starts
    for (int64_t p = 1; p < n; p++)
        if (prank[p] != prank[p - 1]) bnd.push_back(p);
    const std::vector<int64_t> cut = leaf_cuts(bnd, n, t.n_leaves);
    std::vector<int32_t> lf(t.n_leaves), lc(t.n_leaves);
    for (int64_t j = 0; j < t.n_leaves; j++) {
        lf[j] = (int32_t)cut[j];
        lc[j] = (int32_t)(cut[j + 1] - cut[j]);
    }
    upload(t.leaf_first, lf, st);
    upload(t.leaf_cnt, lc, st);
    clock.mark("partition");

    // ---- tables in leaf order -------------------------------------------------
    d.npad = (n + kSlab - 1) / kSlab * kSlab;
    d.n_slabs = d.npad / kSlab;
    d.X32.alloc((size_t)d.npad * dp * sizeof(float));
    GTS_HIP(hipMemsetAsync(d.X32.p, 0, (size_t)d.npad * dp * sizeof(float), st));
    k::gather_rows(in_x.as<float>(), dp, operm.as<int32_t>(), n, d.X32.as<float>(), st);
    d.PT.alloc((size_t)mpad * n * sizeof(float));
    k::gather_pt(pt_in.as<float>(), operm.as<int32_t>(), n, m, mpad, d.PT.as<float>(), st);
    t.box_aos.alloc((size_t)t.n_nodes * 2 * mpad * sizeof(float));
    t.box_lo.alloc((size_t)mpad * t.n_nodes * sizeof(float));
    t.box_hi.alloc((size_t)mpad * t.n_nodes * sizeof(float));
    k::node_boxes(d.PT.as<float>(), n, m, mpad, t.leaf_first.as<int32_t>(), t.leaf_cnt.as<int32_t>(), t.n_leaves,
                  t.leaf0, t.n_nodes, t.fanout, t.levels, t.box_aos.as<float>(), t.box_lo.as<float>(),
                  t.box_hi.as<float>(), st);
    DevBuf ptmax;
    ptmax.alloc(sizeof(uint32_t));
    k::fill_u32(ptmax.as<uint32_t>(), 1, 0u, st);
    k::max_f32(d.PT.as<float>(), (int64_t)m * n, ptmax.as<uint32_t>(), st);
    clock.mark("boxes");
    if (!l1) {
        d.X16t.alloc((size_t)d.npad * d.ksteps * 32 * sizeof(uint16_t));
        d.xn.alloc((size_t)d.npad * sizeof(float));
        d.xe.alloc((size_t)d.npad * sizeof(float));
        k::rows_bf16(d.X32.as<float>(), n, d.npad, d.dim, dp, d.ksteps, d.X16t.as<uint16_t>(), d.xn.as<float>(),
                     d.xe.as<float>(), INFINITY, st);
        d.slab_emax.alloc((size_t)d.n_slabs * sizeof(float));
        d.slab_nmax.alloc((size_t)d.n_slabs * sizeof(float));
        d.slab_leaf_lo.alloc((size_t)d.n_slabs * sizeof(int32_t));
        d.slab_leaf_hi.alloc((size_t)d.n_slabs * sizeof(int32_t));
        k::slab_summary(d.xn.as<float>(), d.xe.as<float>(), n, t.leaf_first.as<int32_t>(), t.n_leaves, d.n_slabs,
                        d.slab_emax.as<float>(), d.slab_nmax.as<float>(), d.slab_leaf_lo.as<int32_t>(),
                        d.slab_leaf_hi.as<int32_t>(), st);
    }
    // leaf pivots: the leaf's object nearest its centroid and the largest
    // distance from it to the leaf's objects (double, widened by 1e-6)
    d.lpad = (t.n_leaves + 63) / 64 * 64;
    DevBuf cen;
    cen.alloc((size_t)t.n_leaves * d.dim * sizeof(double));
    d.PL32.alloc((size_t)d.lpad * dp * sizeof(float));
    d.leafR.alloc((size_t)d.lpad * sizeof(float));
    k::leaf_pivots(d.X32.as<float>(), dp, d.dim, t.leaf_first.as<int32_t>(), t.leaf_cnt.as<int32_t>(), t.n_leaves,
                   d.lpad, cen.as<double>(), d.PL32.as<float>(), d.leafR.as<float>(), st, l1);
    if (!l1) {
        d.PL16t.alloc((size_t)d.lpad * d.ksteps * 32 * sizeof(uint16_t));
        d.pln.alloc((size_t)d.lpad * sizeof(float));
        d.ple.alloc((size_t)d.lpad * sizeof(float));
        k::rows_bf16(d.PL32.as<float>(), d.lpad, d.lpad, d.dim, dp, d.ksteps, d.PL16t.as<uint16_t>(), d.pln.as<float>(),
                     d.ple.as<float>(), INFINITY, st);
        k::mark_empty(t.leaf_cnt.as<int32_t>(), t.n_leaves, d.lpad, d.pln.as<float>(), st);
    }
    uint32_t pm = 0;
    GTS_HIP(hipMemcpyAsync(&pm, ptmax.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GTS_HIP(hipStreamSynchronize(st));
    std::memcpy(&d.pt_max, &pm, sizeof(float));
    clock.mark("layouts + leaf pivots");
}

void build_edit(gts_index *idx, const HostObjects &objs, StageClock &clock, std::vector<int32_t> &perm32)
{
    hipStream_t st = idx->stream;
    IndexData &d = idx->data;
    Tree &t = d.tree;
    const int64_t n = objs.count();
    const int m = d.m, mpad = t.mpad, F = t.fanout;
    // ---- objects on the device in input order (temporary) -----------------
    DevBuf in_chars, in_off, piv_buf, piv_off, dist_buf;
    alphabet_add(idx, objs.chars);
    upload(in_chars, objs.chars, st);
    upload(in_off, objs.offsets, st);

    clock.mark("upload");
    // ---- pivots by farthest-first traversal -------------------------------
    std::vector<float> PTin((size_t)m * n);       // [m][n], input order
    std::vector<float> mind(n, INFINITY);
    std::vector<int64_t> piv(m);
    dist_buf.alloc((size_t)n * sizeof(float));
    uint64_t rng = idx->opts.seed ? idx->opts.seed : 0x2404009660ULL;
    int64_t next = (int64_t)(splitmix64(&rng) % (uint64_t)n);
    for (int i = 0; i < m; i++) {
        piv[i] = next;
        {
            const int64_t a = objs.offsets[next], b = objs.offsets[next + 1];
            std::vector<uint8_t> pc(objs.chars.begin() + a, objs.chars.begin() + b);
            std::vector<int32_t> po{0, (int32_t)(b - a)};
            upload(piv_buf, pc, st);
            upload(piv_off, po, st);
            k::dist_edit_pivots_f32(in_chars.as<uint8_t>(), in_off.as<int64_t>(), n, piv_buf.as<uint8_t>(),
                                    piv_off.as<int32_t>(), 1, 1, dist_buf.as<float>(), 0, 1, idx->lut.as<uint8_t>(),
                                    idx->arows, st);
        }
        float *row = PTin.data() + (size_t)i * n;
        GTS_HIP(hipMemcpyAsync(row, dist_buf.p, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipStreamSynchronize(st));
        float best = -1.f;
        int64_t arg = 0;
        for (int64_t o = 0; o < n; o++) {
            mind[o] = std::min(mind[o], row[o]);
            if (mind[o] > best) {
                best = mind[o];
                arg = o;
            }
        }
        next = arg;
    }

    clock.mark("global pivots + table");
    // ---- leaf order: farthest-first centres, cells, chain, cuts ------------
    // The shape of the tree is fixed (levels, fanout); the partition decides
    // the order of the objects and where each leaf begins.  Every object joins
    // the cell of its nearest farthest-first centre; cells are laid out along
    // a nearest-neighbour chain of their centres and, inside a cell, objects
    // by distance to the centre.  Leaf boundaries start equal-count and each
    // moves to a cell boundary within half a leaf when there is one, so that
    // leaves do not straddle clusters.  A node covers its F children's runs.
    std::vector<int64_t> perm(n);
    std::vector<int64_t> nfirst(t.n_nodes, 0), ncnt(t.n_nodes, 0);
    {
        const int K = (int)std::max<int64_t>(1, std::min<int64_t>({t.n_leaves / 8, (int64_t)kMaxCentres, n}));
        DevBuf d_keys, d_cent, d_mind, d_near, d_cx, d_coff, d_coff32, d_dk;
        std::vector<uint64_t> keys(K + 1, 0ull);
        uint64_t crng = (idx->opts.seed ? idx->opts.seed : 0x2404009660ULL) ^ 0x5bd1e9955bd1e995ULL;
        const int64_t first_centre = (int64_t)(splitmix64(&crng) % (uint64_t)n);
        keys[0] = (uint64_t)(0xffffffffu - (uint32_t)first_centre);
        upload(d_keys, keys, st);
        d_cent.alloc((size_t)K * sizeof(int32_t));
        d_mind.alloc((size_t)n * sizeof(float));
        d_near.alloc((size_t)n * sizeof(int32_t));
        k::fft_centers_edit(in_chars.as<uint8_t>(), in_off.as<int64_t>(), n, idx->lut.as<uint8_t>(), idx->arows,
                                K, d_keys.as<uint64_t>(), d_cent.as<int32_t>(), d_mind.as<float>(),
                                d_near.as<int32_t>(), st);
        std::vector<int32_t> cent(K), nearc(n);
        std::vector<float> cmind(n);
        GTS_HIP(hipMemcpyAsync(cent.data(), d_cent.p, (size_t)K * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipMemcpyAsync(nearc.data(), d_near.p, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipMemcpyAsync(cmind.data(), d_mind.p, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipStreamSynchronize(st));
        clock.mark("centres");
        // centre-to-centre distances, then the chain
        std::vector<float> dk((size_t)K * K);
        d_dk.alloc(dk.size() * sizeof(float));
        std::vector<uint8_t> cc;
        std::vector<int64_t> coff{0};
        {
            for (int c = 0; c < K; c++) {
                cc.insert(cc.end(), objs.chars.begin() + objs.offsets[cent[c]],
                          objs.chars.begin() + objs.offsets[cent[c] + 1]);
                coff.push_back((int64_t)cc.size());
            }
            std::vector<int32_t> coff32(coff.begin(), coff.end());
            if (cc.empty()) cc.push_back(0);
            upload(d_cx, cc, st);
            upload(d_coff, coff, st);
            upload(d_coff32, coff32, st);
            k::dist_edit_pivots_f32(d_cx.as<uint8_t>(), d_coff.as<int64_t>(), K, d_cx.as<uint8_t>(),
                                    d_coff32.as<int32_t>(), K, K, d_dk.as<float>(), K, 1, idx->lut.as<uint8_t>(),
                                    idx->arows, st);
        }
        GTS_HIP(hipMemcpyAsync(dk.data(), d_dk.p, dk.size() * sizeof(float), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipStreamSynchronize(st));
        std::vector<int32_t> rank, by_rank;
        centre_chain(dk, K, rank, by_rank);
        {
            // centre strings in chain order (queries look up their nearest one)
            std::vector<uint8_t> rc;
            std::vector<int32_t> ro{0};
            for (int r = 0; r < K; r++) {
                const int c = by_rank[r];
                rc.insert(rc.end(), objs.chars.begin() + objs.offsets[cent[c]],
                          objs.chars.begin() + objs.offsets[cent[c] + 1]);
                ro.push_back((int32_t)rc.size());
            }
            if (rc.empty()) rc.push_back(0);
            upload(d.cchars, rc, st);
            upload(d.coff, ro, st);
            d.n_centres = K;
            // centre-to-centre distances in chain order (strings of at most
            // kMaxStrlen bytes: every distance fits a byte), and the q-gram
            // buckets of the centre strings (CSR, ranks ascending per bucket)
            std::vector<uint8_t> cdist((size_t)K * K);
            for (int r1 = 0; r1 < K; r1++)
                for (int r2 = 0; r2 < K; r2++) {
                    const float v = dk[(size_t)by_rank[r1] * K + by_rank[r2]];
                    k::require(v >= 0.f && v <= 255.f, "build: centre distance outside 0..255");
                    cdist[(size_t)r1 * K + r2] = (uint8_t)v;
                }
            upload(d.cell_dist, cdist, st);
            std::vector<uint64_t> ent;   // (bucket << 32) | rank
            for (int r = 0; r < K; r++) {
                const int len = ro[r + 1] - ro[r];
                const size_t e0 = ent.size();
                for (int p = 0; p + k::kQgram <= len; p++)
                    ent.push_back(((uint64_t)k::qgram_bucket(rc.data() + ro[r] + p) << 32) | (uint32_t)r);
                std::sort(ent.begin() + e0, ent.end());
                ent.erase(std::unique(ent.begin() + e0, ent.end()), ent.end());
            }
            std::sort(ent.begin(), ent.end());
            std::vector<int32_t> qoff(k::kQgramBuckets + 1, 0), qcell(std::max<size_t>(ent.size(), 1), 0);
            for (size_t e = 0; e < ent.size(); e++) {
                qoff[(ent[e] >> 32) + 1]++;
                qcell[e] = (int32_t)(uint32_t)ent[e];
            }
            for (int b2 = 0; b2 < k::kQgramBuckets; b2++) qoff[b2 + 1] += qoff[b2];
            upload(d.qg_off, qoff, st);
            upload(d.qg_cell, qcell, st);
        }
        std::iota(perm.begin(), perm.end(), 0);
        std::sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) {
            const int32_t rx = rank[nearc[x]], ry = rank[nearc[y]];
            if (rx != ry) return rx < ry;
            if (cmind[x] != cmind[y]) return cmind[x] < cmind[y];
            return objs.ids[x] < objs.ids[y];
        });
        // leaf cuts
        std::vector<int64_t> bnd;   // positions where a new cell starts
        for (int64_t p = 1; p < n; p++)
            if (nearc[perm[p]] != nearc[perm[p - 1]]) bnd.push_back(p);
        const int64_t L = t.n_leaves;
        const std::vector<int64_t> cut = leaf_cuts(bnd, n, L);
        for (int64_t j2 = 0; j2 < L; j2++) {
            nfirst[t.leaf0 + j2] = cut[j2];
            ncnt[t.leaf0 + j2] = cut[j2 + 1] - cut[j2];
        }
        {
            // per cell: covering radius, pivot box and length range; per leaf:
            // the cells it spans
            std::vector<float> cR(K, -INFINITY), cbox((size_t)K * 2 * mpad);
            std::vector<int32_t> clen((size_t)2 * K);
            for (int r = 0; r < K; r++) {
                for (int i = 0; i < mpad; i++) {
                    cbox[(size_t)r * 2 * mpad + i] = i < m ? INFINITY : -INFINITY;
                    cbox[(size_t)r * 2 * mpad + mpad + i] = i < m ? -INFINITY : INFINITY;
                }
                clen[2 * r] = INT32_MAX;
                clen[2 * r + 1] = INT32_MIN;
            }
            for (int64_t p = 0; p < n; p++) {
                const int64_t o = perm[p];
                const int r = rank[nearc[o]];
                cR[r] = std::max(cR[r], cmind[o]);
                float *b = cbox.data() + (size_t)r * 2 * mpad;
                for (int i = 0; i < m; i++) {
                    const float x = PTin[(size_t)i * n + o];
                    b[i] = std::min(b[i], x);
                    b[mpad + i] = std::max(b[mpad + i], x);
                }
                const int32_t len = (int32_t)(objs.offsets[o + 1] - objs.offsets[o]);
                clen[2 * r] = std::min(clen[2 * r], len);
                clen[2 * r + 1] = std::max(clen[2 * r + 1], len);
            }
            std::vector<int32_t> lcell((size_t)2 * L);
            for (int64_t j2 = 0; j2 < L; j2++) {
                if (cut[j2 + 1] > cut[j2]) {
                    lcell[2 * j2] = rank[nearc[perm[cut[j2]]]];
                    lcell[2 * j2 + 1] = rank[nearc[perm[cut[j2 + 1] - 1]]];
                } else {
                    lcell[2 * j2] = 1;
                    lcell[2 * j2 + 1] = 0;
                }
            }
            upload(d.cellR, cR, st);
            upload(d.cell_box, cbox, st);
            upload(d.cell_len, clen, st);
            upload(d.leaf_cell, lcell, st);
            std::vector<int32_t> cleaf((size_t)2 * K);
            for (int r = 0; r < K; r++) {
                cleaf[2 * r] = 1;
                cleaf[2 * r + 1] = 0;
            }
            for (int64_t j2 = L - 1; j2 >= 0; j2--)
                for (int r = lcell[2 * j2]; r <= lcell[2 * j2 + 1]; r++) {
                    if (cleaf[2 * r] > cleaf[2 * r + 1]) cleaf[2 * r + 1] = (int32_t)j2;
                    cleaf[2 * r] = (int32_t)j2;
                }
            upload(d.cell_leaf, cleaf, st);
        }
        for (int64_t v = t.leaf0 - 1; v >= 0; v--) {
            nfirst[v] = nfirst[v * F + 1];
            ncnt[v] = 0;
            for (int c = 0; c < F; c++) ncnt[v] += ncnt[v * F + 1 + c];
        }
    }

    clock.mark("partition");
    // ---- node boxes over every pivot --------------------------------------
    std::vector<float> lo((size_t)t.n_nodes * mpad, INFINITY), hi((size_t)t.n_nodes * mpad, -INFINITY);
    for (int64_t j = 0; j < t.n_leaves; j++) {
        const int64_t v = t.leaf0 + j;
        for (int64_t p = nfirst[v]; p < nfirst[v] + ncnt[v]; p++) {
            const int64_t o = perm[p];
            for (int i = 0; i < m; i++) {
                const float x = PTin[(size_t)i * n + o];
                lo[v * mpad + i] = std::min(lo[v * mpad + i], x);
                hi[v * mpad + i] = std::max(hi[v * mpad + i], x);
            }
        }
    }
    for (int64_t v = t.leaf0 - 1; v >= 0; v--)
        for (int j = 0; j < F; j++) {
            const int64_t c = v * F + 1 + j;
            for (int i = 0; i < m; i++) {
                lo[v * mpad + i] = std::min(lo[v * mpad + i], lo[c * mpad + i]);
                hi[v * mpad + i] = std::max(hi[v * mpad + i], hi[c * mpad + i]);
            }
        }
    for (int64_t v = 0; v < t.n_nodes; v++)
        for (int i = m; i < mpad; i++)
            if (ncnt[v] > 0) {
                lo[v * mpad + i] = -INFINITY;
                hi[v * mpad + i] = INFINITY;
            }
    std::vector<float> aos((size_t)t.n_nodes * 2 * mpad), blo((size_t)mpad * t.n_nodes), bhi((size_t)mpad * t.n_nodes);
    for (int64_t v = 0; v < t.n_nodes; v++)
        for (int i = 0; i < mpad; i++) {
            aos[(size_t)v * 2 * mpad + i] = lo[v * mpad + i];
            aos[(size_t)v * 2 * mpad + mpad + i] = hi[v * mpad + i];
            blo[(size_t)i * t.n_nodes + v] = lo[v * mpad + i];
            bhi[(size_t)i * t.n_nodes + v] = hi[v * mpad + i];
        }
    upload(t.box_aos, aos, st);
    upload(t.box_lo, blo, st);
    upload(t.box_hi, bhi, st);
    std::vector<int32_t> lf(t.n_leaves), lc(t.n_leaves);
    for (int64_t j = 0; j < t.n_leaves; j++) {
        lf[j] = (int32_t)nfirst[t.leaf0 + j];
        lc[j] = (int32_t)ncnt[t.leaf0 + j];
    }
    upload(t.leaf_first, lf, st);
    upload(t.leaf_cnt, lc, st);

    clock.mark("boxes");
    // ---- strings, pivot table in leaf order ---------------------------------
    HostObjects h;   // the strings in leaf order (the host mirror keeps input order)
    h.metric = objs.metric;
    h.dim = objs.dim;
    for (int64_t p = 0; p < n; p++) h.append_from(objs, perm[p]);
    d.pt_max = 0.f;
    for (float x : PTin) d.pt_max = std::max(d.pt_max, x);
    std::vector<int32_t> soff(n + 1);
    for (int64_t p = 0; p <= n; p++) soff[p] = (int32_t)h.offsets[p];
    upload(d.chars, h.chars, st);
    upload(d.soff, soff, st);
    std::vector<uint8_t> pte((size_t)mpad * n, 0), pta((size_t)n * mpad, 0);
    for (int i = 0; i < m; i++)
        for (int64_t p = 0; p < n; p++) {
            const uint8_t v = (uint8_t)PTin[(size_t)i * n + perm[p]];
            pte[(size_t)i * n + p] = v;
            pta[(size_t)p * mpad + i] = v;
        }
    upload(d.PTe, pte, st);
    upload(d.PTa, pta, st);
    std::vector<uint8_t> pc;
    std::vector<int32_t> po{0};
    d.pivot_str.clear();
    for (int i = 0; i < m; i++) {
        const int64_t a = objs.offsets[piv[i]], b = objs.offsets[piv[i] + 1];
        pc.insert(pc.end(), objs.chars.begin() + a, objs.chars.begin() + b);
        po.push_back((int32_t)pc.size());
        d.pivot_str.emplace_back(objs.chars.begin() + a, objs.chars.begin() + b);
    }
    upload(d.pchars, pc, st);
    upload(d.poff, po, st);
    d.npad = n;
    // leaf pivots: the first object of each leaf; R_L from the GPU
    d.lpad = t.n_leaves;
    d.leafR.alloc((size_t)t.n_leaves * sizeof(float));
    k::EditView ev{d.chars.as<uint8_t>(), d.soff.as<int32_t>(), n, idx->lut.as<uint8_t>(), idx->arows};
    k::leaf_radius_edit(ev, t.leaf_first.as<int32_t>(), t.leaf_cnt.as<int32_t>(), t.n_leaves,
                        d.leafR.as<float>(), st);
    GTS_HIP(hipStreamSynchronize(st));
    perm32.assign(perm.begin(), perm.end());
    clock.mark("layouts + leaf pivots");
}

}  // namespace

void build_tree(gts_index *idx, HostObjects &objs, DevBuf *rows)
{
    hipStream_t st = idx->stream;
    IndexData &d = idx->data;
    StageClock clock;
    const int64_t n = objs.count();
    GTS_CHECK(n >= 1, GTS_EINVAL, "an index needs at least one object");
    GTS_CHECK(n < (int64_t)1 << 31, GTS_ENOTSUP, "at most 2^31-1 objects per index");
    d.metric = objs.metric;
    d.n = n;
    d.m = idx->num_pivots;
    tree_shape(idx, n);
    std::vector<int32_t> perm;   // input row of each position
    if (objs.metric == GTS_L2_F32) build_l2(idx, objs, rows, clock, perm);
    else build_edit(idx, objs, clock, perm);

    // ---- ids in leaf order, tombstones, id maps, host mirror ----------------
    std::vector<uint32_t> pid(n);
    uint32_t max_id = 0;
    for (int64_t p = 0; p < n; p++) {
        pid[p] = objs.ids[perm[p]];
        max_id = std::max(max_id, pid[p]);
    }
    upload(d.ids, pid, st);
    const int64_t words = (std::max(d.npad, n) + 31) / 32 + 1;
    d.tomb_words = words;
    d.tomb.alloc((size_t)words * sizeof(uint32_t));
    k::fill_u32(d.tomb.as<uint32_t>(), words, 0u, st);
    d.del_ep.alloc((size_t)words * 32 * sizeof(uint32_t));
    k::fill_u32(d.del_ep.as<uint32_t>(), words * 32, 0xffffffffu, st);
    idx->h_tomb.assign(n, 0);
    idx->n_deleted_tree = 0;
    idx->pos_of_id.assign(std::max<int64_t>((int64_t)max_id + 1, idx->next_id), -1);
    for (int64_t p = 0; p < n; p++) idx->pos_of_id[pid[p]] = p;
    // the host mirror keeps the objects' ids (and an edit index its strings)
    // in input order; host_row[p] is the row of the object at position p.
    // Vector rows live on the device only.
    idx->host = std::move(objs);
    if (d.metric == GTS_L2_F32) {
        idx->host.vecs.clear();
        idx->host.vecs.shrink_to_fit();
    }
    idx->host_row = std::move(perm);
    GTS_HIP(hipStreamSynchronize(st));
    clock.mark("tombstones + maps");
}

// ---------------------------------------------------------------------------
// Streamed updates (Sec. 4.4).
// ---------------------------------------------------------------------------
namespace {

void cache_reserve(gts_index *idx, int64_t need)
{
    CacheList &c = idx->cache;
    if (need <= c.cap) return;
    int64_t cap = std::max<int64_t>(need, std::max<int64_t>(2 * c.cap, 64));
    hipStream_t st = idx->stream;
    const IndexData &d = idx->data;
    auto grow = [&](DevBuf &b, size_t elem) {
        DevBuf nb;
        nb.alloc((size_t)cap * elem);
        GTS_HIP(hipMemsetAsync(nb.p, 0, (size_t)cap * elem, st));
        if (b.p && c.count) GTS_HIP(hipMemcpyAsync(nb.p, b.p, (size_t)c.count * elem, hipMemcpyDeviceToDevice, st));
        GTS_HIP(hipStreamSynchronize(st));
        std::swap(b.p, nb.p);
        std::swap(b.bytes, nb.bytes);
    };
    if (d.metric == GTS_L2_F32) grow(c.X32, (size_t)d.dp * sizeof(float));
    else grow(c.chars, (size_t)kMaxStrlen);
    grow(c.slen, sizeof(int32_t));
    grow(c.ids, sizeof(uint32_t));
    grow(c.ins_ep, sizeof(uint32_t));
    grow(c.del_ep, sizeof(uint32_t));
    if (d.metric != GTS_L2_F32) grow(c.cp, (size_t)d.tree.mpad * sizeof(float));
    c.cap = cap;
}

}  // namespace

bool tree_mostly_deleted(const gts_index *idx, int64_t more)
{
    return 2 * (idx->n_deleted_tree + more) > idx->data.n;
}

static uint32_t next_epoch(gts_index *idx)
{
    GTS_CHECK(idx->epoch < 0xfffffff0u, GTS_ENOTSUP, "update epochs exhausted (2^32 updates on one index)");
    return ++idx->epoch;
}

void insert_objects(gts_index *idx, const HostObjects &objs, int64_t *out_ids)
{
    const int64_t n = objs.count();
    if (n == 0) return;
    GTS_CHECK(idx->next_id + n < ((int64_t)1 << 31), GTS_ENOTSUP, "id space exhausted (ids stay below 2^31)");
    const uint32_t e = next_epoch(idx);
    hipStream_t st = idx->stream;
    CacheList &c = idx->cache;
    const IndexData &d = idx->data;
    cache_reserve(idx, c.count + n);
    HostObjects &ch = idx->cache_host;
    ch.metric = d.metric;
    ch.dim = d.dim;
    std::vector<uint32_t> nid(n);
    std::vector<int32_t> len(n, 0);
    for (int64_t i = 0; i < n; i++) {
        nid[i] = (uint32_t)idx->next_id++;
        if (out_ids) out_ids[i] = nid[i];
    }
    const int64_t s0 = c.count;
    if (d.metric != GTS_L2_F32) alphabet_add(idx, objs.chars);
    if (d.metric == GTS_L2_F32) {
        rows_to_device(c.X32.as<float>() + (size_t)s0 * d.dp, d.dp, objs.vecs.data(), d.dim, n, false, st);
    } else {
        std::vector<uint8_t> slots((size_t)n * kMaxStrlen, 0);
        for (int64_t i = 0; i < n; i++) {
            len[i] = (int32_t)(objs.offsets[i + 1] - objs.offsets[i]);
            std::copy(objs.chars.begin() + objs.offsets[i], objs.chars.begin() + objs.offsets[i + 1],
                      slots.begin() + (size_t)i * kMaxStrlen);
        }
        GTS_HIP(hipMemcpyAsync(c.chars.as<uint8_t>() + (size_t)s0 * kMaxStrlen, slots.data(), slots.size(),
                               hipMemcpyHostToDevice, st));
    }
    GTS_HIP(hipMemcpyAsync(c.slen.as<int32_t>() + s0, len.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st));
    GTS_HIP(hipMemcpyAsync(c.ids.as<uint32_t>() + s0, nid.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    k::fill_u32(c.ins_ep.as<uint32_t>() + s0, n, e, st);
    k::fill_u32(c.del_ep.as<uint32_t>() + s0, n, 0xffffffffu, st);
    // edit distance: the new slots' distances to the global pivots (the
    // cache scan's Lemma 1; for L2 the scan is a dense distance tile)
    if (d.metric != GTS_L2_F32) {
        const int mpad = d.tree.mpad;
        float *cp = c.cp.as<float>() + (size_t)s0 * mpad;
        DevBuf sc, so;
        upload(sc, objs.chars.empty() ? std::vector<uint8_t>(1, 0) : objs.chars, st);
        upload(so, objs.offsets, st);
        k::dist_edit_pivots_f32(sc.as<uint8_t>(), so.as<int64_t>(), n, d.pchars.as<uint8_t>(), d.poff.as<int32_t>(),
                                d.m, mpad, cp, 1, mpad, idx->lut.as<uint8_t>(), idx->arows, st);
    }
    GTS_HIP(hipStreamSynchronize(st));
    if ((int64_t)idx->slot_of_id.size() < idx->next_id) idx->slot_of_id.resize(idx->next_id, -1);
    if ((int64_t)idx->pos_of_id.size() < idx->next_id) idx->pos_of_id.resize(idx->next_id, -1);
    for (int64_t i = 0; i < n; i++) {
        ch.metric = objs.metric;
        ch.dim = objs.dim;
        if (objs.metric != GTS_L2_F32) {   // (vector rows stay on the device)
            ch.chars.insert(ch.chars.end(), objs.chars.begin() + objs.offsets[i],
                            objs.chars.begin() + objs.offsets[i + 1]);
            ch.offsets.push_back((int64_t)ch.chars.size());
        }
        ch.ids.push_back(nid[i]);
        c.h_ids.push_back(nid[i]);
        c.h_live.push_back(1);
        idx->slot_of_id[nid[i]] = s0 + i;
    }
    c.count += n;
    c.n_live += n;
    const int64_t limit = idx->opts.cache_limit > 0 ? idx->opts.cache_limit : 4096;
    if (c.n_live > limit) rebuild(idx);
}

int64_t delete_ids(gts_index *idx, const int64_t *ids, int64_t n, bool upload)
{
    hipStream_t st = idx->stream;
    CacheList &c = idx->cache;
    const uint32_t e = next_epoch(idx);
    int64_t done = 0;
    // the device words this batch changes, applied by scatter launches: the
    // deletion epochs of cache slots and tree positions, and the tombstone
    // words of those positions
    std::vector<uint32_t> slot_at, pos_at, tomb_at;
    for (int64_t i = 0; i < n; i++) {
        const int64_t id = ids[i];
        if (id < 0 || id >= idx->next_id) continue;
        if (id < (int64_t)idx->slot_of_id.size() && idx->slot_of_id[id] >= 0) {
            const int64_t s = idx->slot_of_id[id];
            if (c.h_live[s]) {
                c.h_live[s] = 0;
                c.n_live--;
                slot_at.push_back((uint32_t)s);
                idx->slot_of_id[id] = -1;
                done++;
            }
            continue;
        }
        if (id < (int64_t)idx->pos_of_id.size() && idx->pos_of_id[id] >= 0) {
            const int64_t p = idx->pos_of_id[id];
            if (!idx->h_tomb[p]) {
                idx->h_tomb[p] = 1;
                idx->n_deleted_tree++;
                pos_at.push_back((uint32_t)p);
                tomb_at.push_back((uint32_t)(p >> 5));
                done++;
            }
        }
    }
    if (!upload || (slot_at.empty() && pos_at.empty())) return done;
    std::sort(tomb_at.begin(), tomb_at.end());
    tomb_at.erase(std::unique(tomb_at.begin(), tomb_at.end()), tomb_at.end());
    const IndexData &d = idx->data;
    // [slots | positions | tombstone words | their values]; one transfer
    const size_t ns = slot_at.size(), np = pos_at.size(), nt = tomb_at.size(), na = ns + np + nt;
    std::vector<uint32_t> pack(2 * na);
    std::copy(slot_at.begin(), slot_at.end(), pack.begin());
    std::copy(pos_at.begin(), pos_at.end(), pack.begin() + ns);
    std::copy(tomb_at.begin(), tomb_at.end(), pack.begin() + ns + np);
    std::fill(pack.begin() + na, pack.begin() + na + ns + np, e);
    for (size_t i = 0; i < nt; i++) {
        const int64_t w = tomb_at[i];
        uint32_t bits = 0;
        for (int b = 0; b < 32; b++) {
            const int64_t p = w * 32 + b;
            if (p < d.n && idx->h_tomb[p]) bits |= 1u << b;
        }
        pack[na + ns + np + i] = bits;
    }
    DevBuf &dp = idx->upd_buf;
    dp.alloc(pack.size() * sizeof(uint32_t));
    GTS_HIP(hipMemcpyAsync(dp.p, pack.data(), pack.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    const uint32_t *dpk = dp.as<uint32_t>();
    if (ns) k::scatter_u32(c.del_ep.as<uint32_t>(), dpk, dpk + na, (int64_t)ns, st);
    if (np) k::scatter_u32(d.del_ep.as<uint32_t>(), dpk + ns, dpk + na + ns, (int64_t)np, st);
    if (nt) k::scatter_u32(d.tomb.as<uint32_t>(), dpk + ns + np, dpk + na + ns + np, (int64_t)nt, st);
    GTS_HIP(hipStreamSynchronize(st));
    // a tree that is mostly tombstones is rebuilt from its live objects (its
    // boxes and radii still cover the deleted ones, and a kNN bound window
    // may hold fewer live objects than k)
    if (tree_mostly_deleted(idx) && idx->data.n - idx->n_deleted_tree + c.n_live >= 1) rebuild(idx);
    return done;
}

// Batch updates (Sec. 4.4): for bulk changes the index is reconstructed
// directly instead of going through the cache list.  Deletions are marked,
// the new objects take fresh ids, and one rebuild covers every live object
// of the tree, the cache list and the batch.
void update_batch(gts_index *idx, const HostObjects &ins, const int64_t *del, int64_t n_del, int64_t *out_ids,
                  int64_t *n_deleted)
{
    const int64_t n = ins.count();
    GTS_CHECK(idx->next_id + n < ((int64_t)1 << 31), GTS_ENOTSUP, "id space exhausted (ids stay below 2^31)");
    const int64_t done = delete_ids(idx, del, n_del, false);
    if (n_deleted) *n_deleted = done;
    if ((int64_t)idx->slot_of_id.size() < idx->next_id + n) idx->slot_of_id.resize(idx->next_id + n, -1);
    if ((int64_t)idx->pos_of_id.size() < idx->next_id + n) idx->pos_of_id.resize(idx->next_id + n, -1);
    std::vector<uint32_t> new_ids(n);
    for (int64_t i = 0; i < n; i++) {
        new_ids[i] = (uint32_t)idx->next_id++;
        if (out_ids) out_ids[i] = new_ids[i];
    }
    if (idx->data.metric == GTS_L2_F32) {
        // the new rows join the rebuild on the device
        DevBuf rows;
        rows.alloc((size_t)std::max<int64_t>(n, 1) * idx->data.dp * sizeof(float));
        rows_to_device(rows.as<float>(), idx->data.dp, ins.vecs.data(), ins.dim, n, false, idx->stream);
        rebuild(idx, &rows, n, new_ids.data());
        return;
    }
    HostObjects &ch = idx->cache_host;
    ch.metric = idx->data.metric;
    ch.dim = idx->data.dim;
    for (int64_t i = 0; i < n; i++) {
        ch.chars.insert(ch.chars.end(), ins.chars.begin() + ins.offsets[i], ins.chars.begin() + ins.offsets[i + 1]);
        ch.offsets.push_back((int64_t)ch.chars.size());
        ch.ids.push_back(new_ids[i]);
        idx->cache.h_ids.push_back(new_ids[i]);
        idx->cache.h_live.push_back(1);
    }
    if (n) alphabet_add(idx, ins.chars);
    rebuild(idx);
}

// Rebuild over every live object (Sec. 4.4: when the cache list exceeds its
// limit the whole index is reconstructed from the index and the cache).
void rebuild(gts_index *idx, DevBuf *extra_rows, int64_t n_extra, const uint32_t *extra_ids)
{
    const auto t0 = std::chrono::steady_clock::now();
    HostObjects all;
    all.metric = idx->data.metric;
    all.dim = idx->host.dim ? idx->host.dim : idx->cache_host.dim;
    const HostObjects &h = idx->host;
    const CacheList &cl = idx->cache;
    if (idx->data.metric == GTS_L2_F32) {
        // vector rows never leave the device: the live tree rows, the live
        // cache rows and the batch's new rows are gathered there
        IndexData &d = idx->data;
        hipStream_t st = idx->stream;
        std::vector<int32_t> tree_pos, slots;
        for (int64_t p = 0; p < (int64_t)idx->host_row.size(); p++)
            if (!idx->h_tomb[p]) {
                tree_pos.push_back((int32_t)p);
                all.ids.push_back(h.ids[idx->host_row[p]]);
            }
        for (int64_t s = 0; s < cl.count; s++)
            if (cl.h_live[s]) {
                slots.push_back((int32_t)s);
                all.ids.push_back(cl.h_ids[s]);
            }
        for (int64_t i = 0; i < n_extra; i++) all.ids.push_back(extra_ids[i]);
        const int64_t n = all.count();
        GTS_CHECK(n >= 1, GTS_EINVAL, "cannot rebuild an index with no live objects");
        DevBuf rows, dpos, dslot;
        const size_t row_bytes = (size_t)d.dp * sizeof(float);
        rows.alloc((size_t)n * row_bytes);
        const int64_t a = (int64_t)tree_pos.size(), b = (int64_t)slots.size();
        if (a) {
            upload(dpos, tree_pos, st);
            k::gather_rows(d.X32.as<float>(), d.dp, dpos.as<int32_t>(), a, rows.as<float>(), st);
        }
        if (b) {
            upload(dslot, slots, st);
            k::gather_rows(cl.X32.as<float>(), d.dp, dslot.as<int32_t>(), b, rows.as<float>() + (size_t)a * d.dp,
                           st);
        }
        if (n_extra)
            GTS_HIP(hipMemcpyAsync(rows.as<float>() + (size_t)(a + b) * d.dp, extra_rows->p, (size_t)n_extra * row_bytes,
                                   hipMemcpyDeviceToDevice, st));
        GTS_HIP(hipStreamSynchronize(st));
        build_tree(idx, all, &rows);
    } else {
        for (int64_t p = 0; p < (int64_t)idx->host_row.size(); p++)
            if (!idx->h_tomb[p]) all.append_from(h, idx->host_row[p]);
        const HostObjects &ch = idx->cache_host;
        for (int64_t s = 0; s < ch.count(); s++)
            if (cl.h_live[s]) all.append_from(ch, s);
        GTS_CHECK(all.count() >= 1, GTS_EINVAL, "cannot rebuild an index with no live objects");
        build_tree(idx, all);
    }
    CacheList &c = idx->cache;
    c.count = 0;
    c.n_live = 0;
    c.h_ids.clear();
    c.h_live.clear();
    idx->cache_host.clear();
    std::fill(idx->slot_of_id.begin(), idx->slot_of_id.end(), -1);
    idx->rebuilds++;
    idx->rebuild_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace gts
