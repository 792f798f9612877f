// Sampling (parity hook), initial values, table conversion, kernel dispatch and the
// workspace layouts.
#include "handle.hpp"
#include "scan.hpp"
#include "sgd_kernels.hpp"

namespace lh {

LH_DECLARE_LAUNCHERS(float, 1)
LH_DECLARE_LAUNCHERS(float, 2)
LH_DECLARE_LAUNCHERS(float, 3)
LH_DECLARE_LAUNCHERS(uint16_t, 1)
LH_DECLARE_LAUNCHERS(uint16_t, 2)
LH_DECLARE_LAUNCHERS(uint16_t, 3)

// ---------------------------------------------------------------------------
// Workspace layouts.
// ---------------------------------------------------------------------------
static size_t carve(size_t &off, size_t bytes)
{
    size_t at = off;
    off = lh_align_up(off + bytes, 256);
    return at;
}

WsLayout ws_layout(const lh_params &p, long long n, long long m)
{
    WsLayout L;
    size_t off = 0;
    L.status = carve(off, 256);
    L.tiles = carve(off, 256);
    L.erec = carve(off, sizeof(EdgeRec) * (size_t)(m > 0 ? m : 1));
    L.nrec = carve(off, sizeof(NegRec) * (size_t)(n > 0 ? n : 1));
    L.nheat = carve(off, (size_t)(n > 0 ? n : 1));
    if (uses_shadow(p)) {
        const size_t ntab = p.orders == LH_ORDER12 ? 3 : (p.orders == LH_ORDER2 ? 2 : 1);
        L.shadow_cap = shadow_capacity(n > 0 ? n : 1);
        L.slot = carve(off, 4 * (size_t)(n > 0 ? n : 1));
        L.srows = carve(off, 4 * (size_t)L.shadow_cap);
        L.shadow = carve(off, 4 * (size_t)L.shadow_cap * (size_t)p.d * ntab);
    }
    if (p.mode == LH_SNAPSHOT) {
        long long nord = p.orders == 3 ? 2 : 1;
        long long E = p.batch * nord * (long long)(p.K + 2);
        L.entries = E;
        L.keys0 = carve(off, 4 * (size_t)E);
        L.keys1 = carve(off, 4 * (size_t)E);
        L.vals0 = carve(off, 4 * (size_t)E);
        L.vals1 = carve(off, 4 * (size_t)E);
        L.contrib = carve(off, 4 * (size_t)E * (size_t)p.d);
        L.hist_n = 16 * LH_CDIV(E, RADIX_TILE);
        L.hist = carve(off, 4 * (size_t)L.hist_n);
        long long mx = L.hist_n > E ? L.hist_n : E;
        L.ilev_n = scan_levels_size(mx);
        L.ilev = carve(off, 4 * (size_t)L.ilev_n);
        L.seg = carve(off, 4 * (size_t)(E + 1));
        L.segid = carve(off, 4 * (size_t)(E + 1));
    }
    L.total = off;
    return L;
}

ScratchLayout scratch_layout(long long n, long long m)
{
    ScratchLayout L;
    long long N = n > m ? n : m;
    if (N < 1) N = 1;
    L.N = N;
    size_t off = 0;
    L.wq = carve(off, 8 * (size_t)N);
    L.dx = carve(off, 8 * (size_t)N);
    L.idx = carve(off, 4 * (size_t)N);
    L.lpos = carve(off, 4 * (size_t)N);
    L.deg = carve(off, 4 * (size_t)(n > 0 ? n : 1));
    L.indeg = carve(off, 4 * (size_t)(n > 0 ? n : 1));
    L.cnt = carve(off, 8 * 257);
    L.lev_n = scan_levels_size(N);
    L.lev = carve(off, 8 * (size_t)L.lev_n);
    L.ilev = carve(off, 4 * (size_t)L.lev_n);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// Kernel configurations.
// ---------------------------------------------------------------------------
static int next_pow2(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

static int units_per_row(int dtype, int d) { return dtype == LH_FP32 ? d : d / 2; }

// The natural configuration: four units (16 bytes) per lane, lanes = next power of two.
TileCfg natural_cfg(int dtype, int d)
{
    const int nu = units_per_row(dtype, d);
    TileCfg c;
    c.lps = next_pow2(LH_CDIV(nu, 4));
    if (c.lps < 2) c.lps = 2;
    c.upl = 4;
    if (c.lps > 64) {
        c.lps = 64;
        c.upl = 8;
    }
    c.blocks_per_cu = 8;
    return c;
}

// The Hogwild configuration before any tuning or degrees.  Binary32: the natural one.
// bfloat16 (whose timing runs are switched off): one sample per wavefront, one 4-byte unit
// per lane over up to 64 lanes (wider rows: more units per lane).  auto_cfg may move a
// bfloat16 handle to two samples per wavefront once the degrees are known.
TileCfg default_cfg(int dtype, int d)
{
    if (dtype == LH_FP32) return natural_cfg(dtype, d);
    const int nu = units_per_row(dtype, d);
    TileCfg c;
    c.blocks_per_cu = 16;
    if (nu <= 64) {
        c.lps = next_pow2(nu);
        if (c.lps < 16) c.lps = 16;
        c.upl = 1;
    } else {
        c.lps = 64;
        c.upl = next_pow2(LH_CDIV(nu, 64));
    }
    return c;
}

double hot_touch_share(const unsigned long long *heat_count, int hot_heat, int K)
{
    if (hot_heat < 0) return 0.0;
    if (hot_heat >= 255) return 1.0;
    double touches = 0.0;
    for (int v = 0; v <= hot_heat; ++v) touches += (double)heat_count[v] * std::exp2(-(v + 0.5));
    const double share = touches / (2.0 + K);
    return share < 1.0 ? share : 1.0;
}

double hogwild_in_flight(const GraphDev &g, int dtype, int orders, const TileCfg &c, unsigned long long count,
                         int num_cu)
{
    if (dtype == LH_FP32) {
        if (orders == 1) return hogwild_in_flight_t<float, 1>(g, c, count, num_cu);
        if (orders == 2) return hogwild_in_flight_t<float, 2>(g, c, count, num_cu);
        return hogwild_in_flight_t<float, 3>(g, c, count, num_cu);
    }
    if (orders == 1) return hogwild_in_flight_t<uint16_t, 1>(g, c, count, num_cu);
    if (orders == 2) return hogwild_in_flight_t<uint16_t, 2>(g, c, count, num_cu);
    return hogwild_in_flight_t<uint16_t, 3>(g, c, count, num_cu);
}

TileCfg auto_cfg(const lh_handle *h)
{
    TileCfg one = default_cfg(h->p.dtype, h->p.d);
    if (h->p.dtype != LH_BF16 || h->p.mode != LH_HOGWILD) return one;
    TileCfg two = one;
    two.lps = one.lps / 2;
    two.upl = one.upl * 2;
    if (!cfg_supported(h->p.dtype, h->p.d, two)) return one;
    const GraphDev g = graph_dev(h);
    const double F = hogwild_in_flight(g, h->p.dtype, h->p.orders, two, h->p.total_samples, h->num_cu);
    if (!(F > 0.0)) return one;
    const int hot = hot_heat_for(F + g.resid, g.hot_rate);
    return hot_touch_share(h->heat_count, hot, h->p.K) <= kTwoPerWaveMaxHotShare ? two : one;
}

bool cfg_supported(int dtype, int d, const TileCfg &c)
{
    bool listed = false;
#define LH_CHECK_CFG(L, U) listed = listed || (c.lps == L && c.upl == U);
    LH_CFG_LIST(LH_CHECK_CFG)
#undef LH_CHECK_CFG
    return listed && c.lps * c.upl >= units_per_row(dtype, d) && c.blocks_per_cu >= 1 && c.blocks_per_cu <= 64;
}

hipError_t launch_hogwild(const GraphDev &g, int dtype, int orders, const TileCfg &c, unsigned long long first,
                          unsigned long long end, int num_cu, const ShadowCtx *sc, hipStream_t s)
{
    if (dtype == LH_FP32) {
        if (orders == 1) return launch_hogwild_t<float, 1>(g, c, first, end, num_cu, nullptr, s);
        if (orders == 2) return launch_hogwild_t<float, 2>(g, c, first, end, num_cu, nullptr, s);
        return launch_hogwild_t<float, 3>(g, c, first, end, num_cu, nullptr, s);
    }
    if (orders == 1) return launch_hogwild_t<uint16_t, 1>(g, c, first, end, num_cu, sc, s);
    if (orders == 2) return launch_hogwild_t<uint16_t, 2>(g, c, first, end, num_cu, sc, s);
    return launch_hogwild_t<uint16_t, 3>(g, c, first, end, num_cu, sc, s);
}

// ---------------------------------------------------------------------------
// Sampling: one thread per sample, with the draw functions phase A of the training tile
// uses (draw_slot, load_pair_rec, edge_pick, neg_pick).
// ---------------------------------------------------------------------------
__global__ void k_sample(GraphDev g, unsigned long long first, unsigned long long count, int32_t *u, int32_t *v,
                         int32_t *neg)
{
    unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const unsigned long long s = first + i;
    const SlotDraw de = draw_slot(g, s, 0, slot0_columns(g));
    uint4 r0, r1;
    load_pair_rec(g, s, de.col, de.x1, r0, r1);
    int uu = 0, vv = 0;
    (void)edge_pick(r0, r1, de.x1, uu, vv);
    u[i] = uu;
    v[i] = vv;
    for (int j = 1; j <= g.K; ++j) {
        const SlotDraw dn = draw_slot(g, s, j, g.n);
        const uint4 nr = *reinterpret_cast<const uint4 *>(g.nrec + dn.col);
        int id = 0;
        (void)neg_pick(nr, dn, id);
        neg[i * (unsigned long long)g.K + (j - 1)] = id;
    }
}

void launch_sample(lh_handle *h, unsigned long long first, unsigned long long count, int32_t *u, int32_t *v,
                   int32_t *neg, const int2 *pairs, unsigned long long pairs_first)
{
    GraphDev g = graph_dev(h);
    g.pairs = pairs;
    g.pairs_first = pairs_first;
    g.pool_n = pairs ? h->walk.pool : 0;
    if (count == 0) return;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)LH_CDIV(count, 256)), dim3(256), 0, h->stream, g, first, count, u,
                       v, neg);
}

// ---------------------------------------------------------------------------
// Initial values: element (t, r, c) = word c % 4 of Philox4x64-10 with key
// (seed, 2^32 | graph_id) and counter (r, c / 4, t, 0); value ((x >> 40) - 2^23)
// 2^-24 / d in binary64, rounded once to binary32 (bfloat16: then to nearest even).
// ---------------------------------------------------------------------------
template <typename TT>
__global__ void k_init(TT *X, int t, long long rows, int d, unsigned long long seed, unsigned long long key1)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n4 = (d + 3) / 4;
    if (i >= rows * n4) return;
    // d a power of two (d >= 8): the row and group come from shifts, and the value is formed
    // in binary32. The integer (x >> 40) - 2^23 has at most 24 significant bits and 2^-24 / d
    // is a power of two, so both the binary64 expression and this one are exact and equal
    // bit for bit; the four values of a group are one 16-byte (8-byte) store.
    if ((d & (d - 1)) == 0 && d >= 8 && ((uintptr_t)X % (4 * sizeof(TT))) == 0) {
        const int sh = __builtin_ctz((unsigned)n4);
        const long long r = i >> sh;
        const int c4 = (int)(i & (long long)(n4 - 1));
        const u64x4 x = philox4x64_10(seed, key1, (unsigned long long)r, (unsigned long long)c4, (unsigned long long)t, 0ull);
        const float scale = 0x1p-24f / (float)d;
        float f[4];
        const unsigned long long w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) f[k] = (float)((int)(w[k] >> 40) - 8388608) * scale;
        if constexpr (sizeof(TT) == 4) {
            *reinterpret_cast<float4 *>(X + r * d + c4 * 4) = make_float4(f[0], f[1], f[2], f[3]);
        } else {
            const uint32_t lo = f32_to_bf16_rne(f[0]) | (f32_to_bf16_rne(f[1]) << 16);
            const uint32_t hi = f32_to_bf16_rne(f[2]) | (f32_to_bf16_rne(f[3]) << 16);
            *reinterpret_cast<uint2 *>(X + r * d + c4 * 4) = make_uint2(lo, hi);
        }
        return;
    }
    long long r = i / n4;
    int c4 = (int)(i % n4);
    u64x4 x = philox4x64_10(seed, key1, (unsigned long long)r, (unsigned long long)c4, (unsigned long long)t, 0ull);
    unsigned long long w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int c = c4 * 4 + k;
        if (c >= d) break;
        double val = ((double)((long long)(w[k] >> 40) - 8388608ll) * 0x1p-24) / (double)d;
        float f = (float)val;
        if constexpr (sizeof(TT) == 4)
            X[r * d + c] = f;
        else
            X[r * d + c] = (uint16_t)f32_to_bf16_rne(f);
    }
}

void launch_init(lh_handle *h)
{
    const lh_params &p = h->p;
    unsigned long long key1 = (1ull << 32) | (unsigned long long)(uint32_t)p.graph_id;
    long long work = h->n * ((p.d + 3) / 4);
    for (int t = 0; t < 3; ++t) {
        if (!h->tab[t]) continue;
        if (p.dtype == LH_FP32)
            hipLaunchKernelGGL(k_init<float>, dim3((unsigned)LH_CDIV(work, 256)), dim3(256), 0, h->stream,
                               (float *)h->tab[t], t, h->n, p.d, p.seed, key1);
        else
            hipLaunchKernelGGL(k_init<uint16_t>, dim3((unsigned)LH_CDIV(work, 256)), dim3(256), 0, h->stream,
                               (uint16_t *)h->tab[t], t, h->n, p.d, p.seed, key1);
    }
}

// ---------------------------------------------------------------------------
// Table <-> binary32 buffer.
// ---------------------------------------------------------------------------
template <typename TT>
__global__ void k_rw(TT *X, long long off, long long count, float *buf, int write)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    if (write) {
        if constexpr (sizeof(TT) == 4)
            X[off + i] = buf[i];
        else
            X[off + i] = (uint16_t)f32_to_bf16_rne(buf[i]);
    } else {
        if constexpr (sizeof(TT) == 4)
            buf[i] = X[off + i];
        else
            buf[i] = bf16_bits_to_f32(X[off + i]);
    }
}

void launch_rw(lh_handle *h, int table, long long row0, long long rows, float *buf, bool write)
{
    long long count = rows * h->p.d, off = row0 * h->p.d;
    if (count <= 0) return;
    dim3 grid((unsigned)LH_CDIV(count, 256));
    if (h->p.dtype == LH_FP32)
        hipLaunchKernelGGL(k_rw<float>, grid, dim3(256), 0, h->stream, (float *)h->tab[table], off, count, buf,
                           write ? 1 : 0);
    else
        hipLaunchKernelGGL(k_rw<uint16_t>, grid, dim3(256), 0, h->stream, (uint16_t *)h->tab[table], off, count,
                           buf, write ? 1 : 0);
}

// ---------------------------------------------------------------------------
// bfloat16 Hogwild: the binary32 shadow of the hot rows.
// ---------------------------------------------------------------------------
__global__ void k_zero_u32(unsigned int *p) { *p = 0u; }

// Slot of every node: nodes with heat <= hot (and a nonzero rate) take the next free slot
// below cap, one atomic per wavefront; the others get -1.  The order of the slots is
// immaterial: a slot only says where the row lives during the launch.
__global__ void __launch_bounds__(256) k_shadow_slots(const uint8_t *nheat, long long n, int hot, long long cap,
                                                      unsigned int *counter, int32_t *slot, int32_t *srows)
{
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const unsigned hv = r < n ? (unsigned)nheat[r] : 255u;
    const bool want = r < n && hv != 255u && (int)hv <= hot;
    const unsigned long long mask = __ballot(want);
    unsigned base = 0u;
    if (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        if (lane == leader) base = atomicAdd(counter, (unsigned)__popcll(mask));
        base = (unsigned)__shfl((int)base, leader);
    }
    if (r < n) {
        int sv = -1;
        if (want) {
            const unsigned long long idx = (unsigned long long)base + __popcll(mask & ((1ull << lane) - 1ull));
            if (idx < (unsigned long long)cap) {
                sv = (int)idx;
                srows[idx] = (int32_t)r;
            }
        }
        slot[r] = sv;
    }
}

struct ShadowDev {
    float *shadow[3];
    uint32_t *tab[3];  // the bfloat16 tables as 4-byte units (two values each)
    const int32_t *srows;
    const unsigned int *counter;
    long long cap;
    int d, nunits;
    unsigned long long seed, sr_key, first;
};

// One thread per (slot, unit, table): widen the row into the shadow (even elements of the
// row first, then the odd ones).
__global__ void __launch_bounds__(256) k_shadow_load(ShadowDev a, long long bound)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)a.nunits;
    const long long sl = i / per;
    const int un = (int)(i % per);
    const long long used = (long long)*a.counter < a.cap ? (long long)*a.counter : a.cap;
    if (sl >= bound || sl >= used) return;
    const long long r = a.srows[sl];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (!a.shadow[t]) continue;
        const uint32_t w = a.tab[t][r * per + un];
        float *sw = a.shadow[t] + sl * a.d;  // even elements, then odd ones
        sw[un] = __uint_as_float(w << 16);
        sw[per + un] = __uint_as_float(w & 0xffff0000u);
    }
}

// One thread per (slot, unit, table): round the shadow row back into the table, with
// stochastic rounding whose bits come from Philox4x64-10 keyed by (seed, sr_key) at
// counter (first, table, row, unit / 8), 32 bits per unit.
__global__ void __launch_bounds__(256) k_shadow_store(ShadowDev a, long long bound)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)a.nunits;
    const long long sl = i / per;
    const int un = (int)(i % per);
    const long long used = (long long)*a.counter < a.cap ? (long long)*a.counter : a.cap;
    if (sl >= bound || sl >= used) return;
    const long long r = a.srows[sl];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (!a.shadow[t]) continue;
        const float *sw = a.shadow[t] + sl * a.d;
        const float2 x = make_float2(sw[un], sw[per + un]);
        const u64x4 q = philox4x64_10(a.seed, a.sr_key, a.first, (unsigned long long)t, (unsigned long long)r,
                                      (unsigned long long)(un / 8));
        const int qi = (un % 8) / 2;
        const unsigned long long wd = qi == 0 ? q.x : qi == 1 ? q.y : qi == 2 ? q.z : q.w;
        const uint32_t rnd = (uint32_t)(wd >> (32 * (un % 2)));
        a.tab[t][r * per + un] = bf16x2_sr(x.x, x.y, rnd);
    }
}

bool shadow_ctx(const lh_handle *h, ShadowCtx *o)
{
    if (!uses_shadow(h->p) || h->lay.shadow_cap <= 0 || !h->ws) return false;
    o->nheat = (const uint8_t *)(h->ws + h->lay.nheat);
    o->slot = (int32_t *)(h->ws + h->lay.slot);
    o->srows = (int32_t *)(h->ws + h->lay.srows);
    long long k = 0;
    for (int t = 0; t < 3; ++t) {
        o->tab[t] = h->tab[t];
        o->shadow[t] = h->tab[t] ? (float *)(h->ws + h->lay.shadow) + k++ * h->lay.shadow_cap * (long long)h->p.d
                                 : nullptr;
    }
    o->counter = (unsigned int *)(h->ws + h->lay.status + 128);
    o->heat_count = h->heat_count;
    o->n = h->n;
    o->cap = h->lay.shadow_cap;
    o->d = h->p.d;
    o->seed = h->p.seed;
    o->sr_key = (3ull << 32) | (unsigned long long)(uint32_t)h->p.graph_id;
    return true;
}

static ShadowDev shadow_dev(const ShadowCtx &sc, unsigned long long first)
{
    ShadowDev a;
    for (int t = 0; t < 3; ++t) {
        a.shadow[t] = sc.shadow[t];
        a.tab[t] = (uint32_t *)sc.tab[t];
    }
    a.srows = sc.srows;
    a.counter = sc.counter;
    a.cap = sc.cap;
    a.d = sc.d;
    a.nunits = sc.d / 2;
    a.seed = sc.seed;
    a.sr_key = sc.sr_key;
    a.first = first;
    return a;
}

// Hot nodes the shadow will hold for threshold hot (an upper bound when the heat counts
// exceed cap at hot = 0, e.g. after an alias import: then the first cap nodes to ask get
// a slot).  The threshold is lowered until the hot set fits.
static long long shadow_rows(const ShadowCtx &sc, int &hot)
{
    if (hot > 254) hot = 254;
    for (;;) {
        long long c = 0;
        for (int v = 0; v <= hot; ++v) c += (long long)sc.heat_count[v];
        if (hot < 0) return 0;
        if (c <= sc.cap || hot == 0) return c < sc.cap ? c : sc.cap;
        --hot;
    }
}

hipError_t shadow_begin(const ShadowCtx &sc, int hot_heat, hipStream_t s)
{
    int hot = hot_heat;
    const long long rows = shadow_rows(sc, hot);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, sc.counter);
    hipLaunchKernelGGL(k_shadow_slots, dim3((unsigned)LH_CDIV(sc.n, 256)), dim3(256), 0, s, sc.nheat, sc.n, hot,
                       sc.cap, sc.counter, sc.slot, sc.srows);
    if (rows > 0)
        hipLaunchKernelGGL(k_shadow_load, dim3((unsigned)LH_CDIV(rows * (sc.d / 2), 256)), dim3(256), 0, s,
                           shadow_dev(sc, 0), rows);
    return hipGetLastError();
}

hipError_t shadow_end(const ShadowCtx &sc, int hot_heat, unsigned long long first, hipStream_t s)
{
    int hot = hot_heat;
    const long long rows = shadow_rows(sc, hot);
    if (rows > 0)
        hipLaunchKernelGGL(k_shadow_store, dim3((unsigned)LH_CDIV(rows * (sc.d / 2), 256)), dim3(256), 0, s,
                           shadow_dev(sc, first), rows);
    return hipGetLastError();
}

}  // namespace lh
