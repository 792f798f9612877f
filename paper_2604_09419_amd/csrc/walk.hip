// Random-walk positive pairs (Sec. IV-B: Algorithm 2, RandomWalk, and Algorithm 3,
// GeneratePairs) on one GPU, where every vertex is local: the walks never stop at a
// remote vertex (the paper's "Local" variant over the whole graph).  Built with
// -ffp-contract=off: the per-row alias tables are binary64 and bitwise reproducible.
//
// Walk graph: the undirected graph of the arcs.  Entry e < m is arc e forwards (tail
// src[e], head dst[e]), entry m + e arc e backwards; both weigh w[e].  Row x (the
// neighbourhood N(x)) lists the entries with tail x in increasing entry index: a stable
// radix sort of the entries by tail.  discrete(N(x)) is the alias table of the row's
// weights, built exactly as the edge and negative tables are (alias.hip) but per row:
// the canonical scans restart at every row (segscan.hpp), and items are numbered within
// the row.
//
// Walk k: Philox4x64-10 key (seed, 5 * 2^32 | graph_id).  Block (k, 0, 0, 0) draws the
// root arc from the edge table (Algorithm 3's weight-normalised edge distribution):
// w_0 = its tail, w_1 = its head.  Block (k, t, 0, 0), t = 1 .. L - 2, draws w_{t+1}
// from row w_t.  A walk visits L vertices (Algorithm 2 counts visited vertices, root
// pair included, up to the walk length).  Pairs: (w_i, w_{i+delta}), delta = 1 .. W - 1
// (window W; W = 2 gives the consecutive pairs Algorithm 2 collects), numbered
// p = sum_{delta' < delta} (L - delta') + i.  Sample order (Algorithm 3 shuffles a
// batch's pairs): sample s = b Bw P + p Bw + j is pair p of walk b Bw + j.
#include <algorithm>
#include <cmath>

#include "handle.hpp"
#include "scan.hpp"
#include "segscan.hpp"
#include "tile.hpp"

#pragma clang fp contract(off)

namespace lh {

constexpr unsigned long long kWalkTag = 5ull;
constexpr int kWalkMaxWindow = 8;
constexpr int kWalkMaxLength = 4096;
// Pairs one buffer fill aims at (the chunk holds whole walk batches).
constexpr long long kWalkChunkPairs = 1ll << 24;

static size_t carve(size_t &off, size_t bytes)
{
    size_t at = off;
    off = lh_align_up(off + bytes, 256);
    return at;
}

WalkLayout walk_layout(long long n, long long m, int L, int W, long long Bw)
{
    WalkLayout w;
    w.P = 0;
    for (int dl = 1; dl < W; ++dl) w.P += L - dl;
    const long long per = Bw * w.P;
    const long long batches = per >= kWalkChunkPairs ? 1 : kWalkChunkPairs / per;
    w.chunk_walks = Bw * batches;
    size_t off = 0;
    w.off = carve(off, 8 * (size_t)(n + 1));
    w.rec = carve(off, sizeof(WalkRec) * (size_t)(2 * m > 0 ? 2 * m : 1));
    w.pairs = carve(off, 8 * (size_t)w.chunk_walks * (size_t)w.P);
    w.total = off;
    return w;
}

namespace {

struct WalkScratch {
    size_t k0, v0, k1, v1, s0, q, hist, ilev, sstart, slen, arena, total;
    long long E, hist_n, ilev_n;
    size_t arena_bytes;
};

WalkScratch walk_scratch_layout(long long n, long long m)
{
    WalkScratch L;
    const long long E = 2 * m > 0 ? 2 * m : 1;
    L.E = E;
    size_t off = 0;
    L.k0 = carve(off, 4 * (size_t)E);
    L.v0 = carve(off, 4 * (size_t)E);
    L.k1 = carve(off, 4 * (size_t)E);
    L.v1 = carve(off, 4 * (size_t)E);
    L.s0 = carve(off, 8 * (size_t)E);
    L.q = carve(off, 8 * (size_t)E);
    L.hist_n = 16 * LH_CDIV(E, RADIX_TILE);
    L.hist = carve(off, 4 * (size_t)L.hist_n);
    L.ilev_n = scan_levels_size(std::max(L.hist_n, E));
    L.ilev = carve(off, 4 * (size_t)L.ilev_n);
    L.sstart = carve(off, 8 * (size_t)(2 * n));
    L.slen = carve(off, 8 * (size_t)(2 * n));
    L.arena_bytes = std::max(seg_scan_bytes(n, E), seg_scan_bytes(2 * n, E));
    L.arena = carve(off, L.arena_bytes);
    L.total = off;
    return L;
}

// Head of entry e.
__device__ __forceinline__ int32_t entry_head(const int32_t *src, const int32_t *dst, long long m, uint32_t e)
{
    return (long long)e < m ? dst[e] : src[(long long)e - m];
}

__device__ __forceinline__ float entry_weight(const float *w, long long m, uint32_t e)
{
    return (long long)e < m ? w[e] : w[(long long)e - m];
}

}  // namespace

// ---------------------------------------------------------------------------
// Rows of the walk graph.
// ---------------------------------------------------------------------------
__global__ void k_walk_keys(const int32_t *src, const int32_t *dst, long long m, uint32_t *keys, uint32_t *vals)
{
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * m) return;
    keys[e] = (uint32_t)(e < m ? src[e] : dst[e - m]);
    vals[e] = (uint32_t)e;
}

// off[x] = the first sorted position whose tail is >= x; off[n] = E.
__global__ void k_row_offsets(const uint32_t *ks, long long E, long long n, long long *off)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    const long long k = ks[i];
    const long long prev = i == 0 ? -1 : (long long)ks[i - 1];
    for (long long x = prev + 1; x <= k; ++x) off[x] = i;
    if (i == E - 1)
        for (long long x = k + 1; x <= n; ++x) off[x] = E;
}

__global__ void k_rows(const long long *off, long long n, long long *start, long long *len)
{
    long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    start[x] = off[x];
    len[x] = off[x + 1] - off[x];
}

__global__ void k_entry_weights(const uint32_t *vs, long long E, const float *w, long long m, double *s0)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < E) s0[i] = (double)entry_weight(w, m, vs[i]);
}

// q = fl(fl(w len) / W) with W the row's scanned total; a row whose total is not a
// positive finite number makes every item heavy (prob 1, itself).  Light flag into lpos.
__global__ void k_row_normalise(const uint32_t *ks, const uint32_t *vs, const long long *off, const double *scan,
                                const float *w, long long m, long long E, double *q, uint32_t *lpos)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    const long long x = ks[i], lo = off[x], hi = off[x + 1];
    const double W = scan[hi - 1];
    const bool ok = W > 0.0 && !isinf(W);
    const double qi = ok ? __ddiv_rn(__dmul_rn((double)entry_weight(w, m, vs[i]), (double)(hi - lo)), W) : 1.0;
    q[i] = qi;
    lpos[i] = qi < 1.0 ? 1u : 0u;
}

// Lights of row x to [lo, lo + nL) and heavies to [lo + nL, hi), each in index order.
// incl: the inclusive count of lights over all positions.
__global__ void k_row_split(const uint32_t *ks, const long long *off, const double *q, const uint32_t *incl,
                            long long E, double *dx, int32_t *idx)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    const long long x = ks[i], lo = off[x];
    const long long base = lo > 0 ? (long long)incl[lo - 1] : 0;
    const long long nL = (long long)incl[off[x + 1] - 1] - base;
    const double qi = q[i];
    if (qi < 1.0) {
        const long long a = (long long)incl[i] - base - 1;
        dx[lo + a] = __dsub_rn(1.0, qi);
        idx[lo + a] = (int32_t)(i - lo);
    } else {
        const long long k = (i - lo) - ((long long)incl[i] - base);
        dx[lo + nL + k] = __dsub_rn(qi, 1.0);
        idx[lo + nL + k] = (int32_t)(i - lo);
    }
}

// Sub-rows: lights of x at 2x, heavies at 2x + 1.
__global__ void k_subrows(const long long *off, const uint32_t *incl, long long n, long long *start, long long *len)
{
    long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const long long lo = off[x], hi = off[x + 1];
    long long nL = 0;
    if (hi > lo) nL = (long long)incl[hi - 1] - (lo > 0 ? (long long)incl[lo - 1] : 0);
    start[2 * x] = lo;
    len[2 * x] = nL;
    start[2 * x + 1] = lo + nL;
    len[2 * x + 1] = hi - lo - nL;
}

__device__ __forceinline__ unsigned long long walk_thr(double prob)
{
    if (prob >= 1.0) return ~0ull;
    return (unsigned long long)__dmul_rn(prob, 18446744073709551616.0);
}

__device__ __forceinline__ long long walk_count_le(const double *X, long long nH, double s)
{
    long long lo = 0, hi = nH;
    while (lo < hi) {
        long long mid = lo + (hi - lo) / 2;
        if (X[mid] <= s)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ long long walk_count_start_lt(const double *D, long long nL, double x)
{
    if (nL == 0 || !(0.0 < x)) return 0;
    long long lo = 0, hi = nL - 1;
    while (lo < hi) {
        long long mid = lo + (hi - lo) / 2;
        if (D[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return 1 + lo;
}

// The closed form of the sweeping construction (alias.hip) within row x, for the item at
// sorted position j of the light/heavy split.  Writes the item's record.
__global__ void k_row_records(const uint32_t *ks, const uint32_t *vs, const long long *off, const uint32_t *incl,
                              const double *q, const double *dx, const int32_t *idx, long long E,
                              const int32_t *src, const int32_t *dst, long long m, WalkRec *rec)
{
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= E) return;
    const long long x = ks[j], lo = off[x], hi = off[x + 1], len = hi - lo;
    const long long base = lo > 0 ? (long long)incl[lo - 1] : 0;
    const long long nL = (long long)incl[hi - 1] - base, nH = len - nL;
    const double *D = dx + lo, *X = dx + lo + nL;
    const int32_t *I = idx + lo;
    const long long a = j - lo;
    const long long item = I[a];
    unsigned long long thr = ~0ull;
    long long al = item;
    if (a < nL) {
        if (nH > 0) {
            const double S = a == 0 ? 0.0 : D[a - 1];
            long long k = walk_count_le(X, nH, S);
            if (k > nH - 1) k = nH - 1;
            thr = walk_thr(q[lo + item]);
            al = I[nL + k];
        }
    } else {
        const long long k = a - nL;
        if (k < nH - 1) {
            const long long jj = walk_count_start_lt(D, nL, X[k]) - 1;
            double ov = 0.0;
            if (jj >= 0) {
                ov = __dsub_rn(D[jj], X[k]);
                if (ov < 0.0) ov = 0.0;
            }
            if (ov > 0.0) {
                const double p = __dsub_rn(1.0, ov);
                thr = walk_thr(p < 0.0 ? 0.0 : p);
                al = I[nL + k + 1];
            }
        }
    }
    WalkRec r;
    r.thr = thr;
    r.keep = entry_head(src, dst, m, vs[lo + item]);
    r.alias = entry_head(src, dst, m, vs[lo + al]);
    rec[lo + item] = r;
}

// ---------------------------------------------------------------------------
// Walks: one thread per walk of a chunk.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_walk(const EdgeRec *erec, long long m, const long long *off,
                                              const WalkRec *rec, unsigned long long seed, unsigned long long key1,
                                              int L, int W, long long Bw, long long P, unsigned long long k0,
                                              long long nwalks, int2 *pairs)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nwalks) return;
    const unsigned long long k = k0 + (unsigned long long)t;
    int2 *out = pairs + (t / Bw) * Bw * P + (t % Bw);
    const u64x4 x0 = philox4x64_10(seed, key1, k, 0ull, 0ull, 0ull);
    uint4 r0, r1;
    load_edge_rec(erec, draw_column(x0.x, m), r0, r1);
    int u = 0, v = 0;
    (void)edge_pick(r0, r1, x0.y, u, v);
    // ring of the last W - 1 vertices: ring[pos % (W - 1)] holds w_pos
    int ring[kWalkMaxWindow - 1];
    ring[0] = u;
    out[0] = make_int2(u, v);  // pair (w_0, w_1): delta 1, i 0
    int cur = v;
    if (W > 2) ring[1 % (W - 1)] = v;
    for (int pos = 2; pos < L; ++pos) {
        const u64x4 x = philox4x64_10(seed, key1, k, (unsigned long long)(pos - 1), 0ull, 0ull);
        const long long lo = off[cur], len = off[cur + 1] - lo;
        int nxt = cur;  // a row without entries is never reached (every step leaves along an entry)
        if (len > 0) {
            const WalkRec r = rec[lo + draw_column(x.x, len)];
            nxt = x.y < r.thr ? r.keep : r.alias;
        }
        // pairs (w_{pos - delta}, w_pos), delta = 1 .. min(W - 1, pos)
        long long pbase = 0;
        for (int dl = 1; dl < W && dl <= pos; ++dl) {
            const int prev = dl == 1 ? cur : ring[(pos - dl) % (W - 1)];
            out[(pbase + pos - dl) * Bw] = make_int2(prev, nxt);
            pbase += L - dl;
        }
        if (W > 2) ring[pos % (W - 1)] = nxt;
        cur = nxt;
    }
}

__global__ void k_pairs_out(const int2 *pairs, long long from, long long count, int32_t *u, int32_t *v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int2 p = pairs[from + i];
    u[i] = p.x;
    v[i] = p.y;
}

__global__ void k_walk_export(const WalkRec *rec, long long E, unsigned long long *thr, int32_t *keep, int32_t *alias)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    const WalkRec r = rec[i];
    thr[i] = r.thr;
    keep[i] = r.keep;
    alias[i] = r.alias;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static lh_status walk_args_ok(long long n, long long m, int L, int W, long long Bw)
{
    if (n < 1 || m < 1 || 2 * m >= (1ll << 32) || n >= (1ll << 31)) return LH_ERR_INVALID_ARG;
    if (L < 2 || L > kWalkMaxLength || W < 2 || W > kWalkMaxWindow || W > L) return LH_ERR_INVALID_ARG;
    if (Bw < 1 || Bw > (1ll << 24)) return LH_ERR_INVALID_ARG;
    long long P = 0;
    for (int dl = 1; dl < W; ++dl) P += L - dl;
    if (Bw * P > (1ll << 27)) return LH_ERR_INVALID_ARG;
    return LH_OK;
}

static lh_status build_walk(lh_handle *h, char *persist, char *scratch, const WalkLayout &WL, const WalkScratch &S)
{
    hipStream_t st = h->stream;
    const long long n = h->n, m = h->m, E = 2 * m;
    WalkState &w = h->walk;
    w.off = (long long *)(persist + WL.off);
    w.rec = (WalkRec *)(persist + WL.rec);
    w.pairs = (int2 *)(persist + WL.pairs);
    uint32_t *k0 = (uint32_t *)(scratch + S.k0), *v0 = (uint32_t *)(scratch + S.v0);
    uint32_t *k1 = (uint32_t *)(scratch + S.k1), *v1 = (uint32_t *)(scratch + S.v1);
    double *s0 = (double *)(scratch + S.s0), *q = (double *)(scratch + S.q);
    uint32_t *hist = (uint32_t *)(scratch + S.hist), *ilev = (uint32_t *)(scratch + S.ilev);
    long long *sstart = (long long *)(scratch + S.sstart), *slen = (long long *)(scratch + S.slen);
    Arena ar;
    ar.base = scratch + S.arena;
    ar.bytes = S.arena_bytes;
    const dim3 blk(256), ge((unsigned)LH_CDIV(E, 256)), gn((unsigned)LH_CDIV(n, 256));

    hipLaunchKernelGGL(k_walk_keys, ge, blk, 0, st, h->src, h->dst, m, k0, v0);
    int bits = 1;
    while (bits < 31 && (1ll << bits) < n) ++bits;
    uint32_t *ks = nullptr, *vs = nullptr;
    radix_sort_u32(k0, v0, k1, v1, E, bits, hist, ilev, st, &ks, &vs);
    // the other pair of sort buffers: light counts and the split's item indices
    uint32_t *incl = ks == k0 ? k1 : k0;
    int32_t *idx = (int32_t *)(vs == v0 ? v1 : v0);

    hipLaunchKernelGGL(k_row_offsets, ge, blk, 0, st, ks, E, n, w.off);
    hipLaunchKernelGGL(k_rows, gn, blk, 0, st, w.off, n, sstart, slen);
    hipLaunchKernelGGL(k_entry_weights, ge, blk, 0, st, vs, E, h->w, m, s0);
    hipError_t e = seg_scan<OpNeumaier>(s0, E, sstart, slen, n, ar, st);
    if (e != hipSuccess) return hip_fail(h, e, "walk rows: weight scan");
    hipLaunchKernelGGL(k_row_normalise, ge, blk, 0, st, ks, vs, w.off, s0, h->w, m, E, q, incl);
    chunk_scan<OpAdd<uint32_t>>(incl, incl, E, ilev, st);
    hipLaunchKernelGGL(k_row_split, ge, blk, 0, st, ks, w.off, q, incl, E, s0, idx);
    hipLaunchKernelGGL(k_subrows, gn, blk, 0, st, w.off, incl, n, sstart, slen);
    e = seg_scan<OpNeumaier>(s0, E, sstart, slen, 2 * n, ar, st);
    if (e == hipSuccess) e = seg_scan<OpMax>(s0, E, sstart, slen, 2 * n, ar, st);
    if (e != hipSuccess) return hip_fail(h, e, "walk rows: deficit and excess scans");
    hipLaunchKernelGGL(k_row_records, ge, blk, 0, st, ks, vs, w.off, incl, q, s0, idx, E, h->src, h->dst, m, w.rec);
    e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "walk rows");
    return LH_OK;
}

static hipError_t generate_chunk(lh_handle *h, long long chunk)
{
    const WalkState &w = h->walk;
    const unsigned long long k0 = (unsigned long long)chunk * (unsigned long long)w.chunk_walks;
    const unsigned long long key1 = (kWalkTag << 32) | (unsigned long long)(uint32_t)h->p.graph_id;
    hipLaunchKernelGGL(k_walk, dim3((unsigned)LH_CDIV(w.chunk_walks, 256)), dim3(256), 0, h->stream, h->erec, h->m,
                       w.off, w.rec, h->p.seed, key1, w.L, w.W, w.Bw, w.P, k0, w.chunk_walks, w.pairs);
    return hipGetLastError();
}

lh_status walk_each_chunk(lh_handle *h, unsigned long long first, unsigned long long count,
                          const std::function<lh_status(unsigned long long, unsigned long long, const int2 *,
                                                        unsigned long long)> &body)
{
    WalkState &w = h->walk;
    if (w.pool > 0) {
        // Pair pool: the collected pairs are chunk 0's first R; every sample draws from them.
        if (w.loaded != 0) {
            w.loaded = -1;
            hipError_t e = generate_chunk(h, 0);
            if (e != hipSuccess) return hip_fail(h, e, "walk generation");
            w.loaded = 0;
        }
        return count > 0 ? body(first, count, w.pairs, 0) : LH_OK;
    }
    const unsigned long long cs = (unsigned long long)w.chunk_walks * (unsigned long long)w.P;
    const unsigned long long end = first + count;
    for (unsigned long long s = first; s < end;) {
        const unsigned long long c = s / cs, c0 = c * cs;
        const unsigned long long stop = std::min(end, c0 + cs);
        if (w.loaded != (long long)c) {
            w.loaded = -1;
            hipError_t e = generate_chunk(h, (long long)c);
            if (e != hipSuccess) return hip_fail(h, e, "walk generation");
            w.loaded = (long long)c;
        }
        lh_status st = body(s, stop - s, w.pairs, c0);
        if (st != LH_OK) return st;
        s = stop;
    }
    return LH_OK;
}

}  // namespace lh

using namespace lh;

extern "C" {

lh_status lh_walk_size(int64_t n, int64_t m, int32_t walk_length, int32_t window, int64_t walks_per_batch,
                       size_t *persist, size_t *scratch)
{
    if (!persist || !scratch) return LH_ERR_INVALID_ARG;
    lh_status st = walk_args_ok(n, m, walk_length, window, walks_per_batch);
    if (st != LH_OK) return st;
    *persist = walk_layout(n, m, walk_length, window, walks_per_batch).total;
    *scratch = walk_scratch_layout(n, m).total;
    return LH_OK;
}

lh_status lh_walk_build(lh_handle *h, int32_t walk_length, int32_t window, int64_t walks_per_batch, void *persist,
                        size_t persist_bytes, void *scratch, size_t scratch_bytes)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->graph_set || !h->edge_ready) return fail(h, LH_ERR_NOT_BUILT, "lh_set_graph and lh_build_alias first");
    if (walk_args_ok(h->n, h->m, walk_length, window, walks_per_batch) != LH_OK)
        return fail(h, LH_ERR_INVALID_ARG, "walk length, window or walks per batch out of range");
    if (!persist || ((uintptr_t)persist & 255u) || !scratch || ((uintptr_t)scratch & 255u))
        return fail(h, LH_ERR_INVALID_ARG, "walk memory must be 256-byte aligned device memory");
    const WalkLayout WL = walk_layout(h->n, h->m, walk_length, window, walks_per_batch);
    const WalkScratch S = walk_scratch_layout(h->n, h->m);
    if (persist_bytes < WL.total || scratch_bytes < S.total)
        return fail(h, LH_ERR_WORKSPACE_TOO_SMALL, "walk memory smaller than lh_walk_size");
    if (h->p.mode == LH_SNAPSHOT && ((unsigned long long)walks_per_batch * (unsigned long long)WL.P) %
                                            (unsigned long long)h->p.batch != 0)
        return fail(h, LH_ERR_INVALID_ARG, "SNAPSHOT with walk pairs needs the batch to divide a walk batch's pairs");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != h->device) (void)hipSetDevice(h->device);
    WalkState &w = h->walk;
    w = WalkState();
    w.L = walk_length;
    w.W = window;
    w.Bw = walks_per_batch;
    w.P = WL.P;
    w.chunk_walks = WL.chunk_walks;
    lh_status st = build_walk(h, (char *)persist, (char *)scratch, WL, S);
    w.ready = st == LH_OK;
    w.loaded = -1;
    if (prev >= 0 && prev != h->device) (void)hipSetDevice(prev);
    return st;
}

lh_status lh_walk_detach(lh_handle *h)
{
    if (!h) return LH_ERR_INVALID_ARG;
    h->walk = WalkState();
    return LH_OK;
}

lh_status lh_walk_pool_size(uint64_t total_samples, uint64_t *pairs)
{
    if (!pairs || total_samples == 0) return LH_ERR_INVALID_ARG;
    // least R >= 2 with R (R - 1) / 2 >= T: start from the binary64 root and correct it
    unsigned long long R = (unsigned long long)std::ceil(0.5 * (1.0 + std::sqrt(1.0 + 8.0 * (double)total_samples)));
    if (R < 2) R = 2;
    auto tri = [](unsigned long long r) { return (unsigned __int128)r * (unsigned __int128)(r - 1) / 2; };
    while (R > 2 && tri(R - 1) >= (unsigned __int128)total_samples) --R;
    while (tri(R) < (unsigned __int128)total_samples) ++R;
    *pairs = R;
    return LH_OK;
}

lh_status lh_walk_pool(lh_handle *h, uint64_t pairs)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->walk.ready) return fail(h, LH_ERR_NOT_BUILT, "lh_walk_build first");
    WalkState &w = h->walk;
    const unsigned long long cap = (unsigned long long)w.chunk_walks * (unsigned long long)w.P;
    if (pairs > cap) return fail(h, LH_ERR_OUT_OF_RANGE, "pool larger than the walk pair buffer");
    w.pool = pairs;
    if (pairs == 0) return LH_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != h->device) (void)hipSetDevice(h->device);
    lh_status st = LH_OK;
    if (w.loaded != 0) {
        w.loaded = -1;
        hipError_t e = generate_chunk(h, 0);
        if (e != hipSuccess) {
            w.pool = 0;
            st = hip_fail(h, e, "walk generation");
        } else {
            w.loaded = 0;
        }
    }
    if (prev >= 0 && prev != h->device) (void)hipSetDevice(prev);
    return st;
}

lh_status lh_walk_pairs(lh_handle *h, uint64_t first, uint64_t count, int32_t *u, int32_t *v)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->walk.ready) return fail(h, LH_ERR_NOT_BUILT, "lh_walk_build first");
    if (h->walk.pool > 0) return fail(h, LH_ERR_UNSUPPORTED, "a pair pool is on: lh_sample gives its pairs");
    if (count > 0 && (!u || !v)) return fail(h, LH_ERR_INVALID_ARG, "NULL output");
    if (first + count < first || count >= (1ull << 40)) return fail(h, LH_ERR_INVALID_ARG, "sample range out of range");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != h->device) (void)hipSetDevice(h->device);
    lh_status st = walk_each_chunk(h, first, count,
                                   [&](unsigned long long sf, unsigned long long sc, const int2 *pairs,
                                       unsigned long long pf) -> lh_status {
                                       const unsigned long long o = sf - first;
                                       hipLaunchKernelGGL(k_pairs_out, dim3((unsigned)LH_CDIV(sc, 256)), dim3(256), 0,
                                                          h->stream, pairs, (long long)(sf - pf), (long long)sc, u + o,
                                                          v + o);
                                       hipError_t e = hipGetLastError();
                                       return e == hipSuccess ? LH_OK : hip_fail(h, e, "walk pairs");
                                   });
    if (prev >= 0 && prev != h->device) (void)hipSetDevice(prev);
    return st;
}

lh_status lh_walk_export(lh_handle *h, int64_t *offsets, uint64_t *thr, int32_t *keep, int32_t *alias)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->walk.ready) return fail(h, LH_ERR_NOT_BUILT, "lh_walk_build first");
    if (!offsets || !thr || !keep || !alias) return fail(h, LH_ERR_INVALID_ARG, "NULL output");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != h->device) (void)hipSetDevice(h->device);
    const long long E = 2 * h->m;
    hipError_t e = hipMemcpyAsync(offsets, h->walk.off, 8 * (size_t)(h->n + 1), hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_walk_export, dim3((unsigned)LH_CDIV(E, 256)), dim3(256), 0, h->stream, h->walk.rec, E,
                           (unsigned long long *)thr, keep, alias);
        e = hipStreamSynchronize(h->stream);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (prev >= 0 && prev != h->device) (void)hipSetDevice(prev);
    return e == hipSuccess ? LH_OK : hip_fail(h, e, "walk export");
}

}  // extern "C"
