// SNAPSHOT mode: a deterministic form of the batch update of Eq. (4).
//
// For batch [b0, b1) every sample's increments are computed from the tables as they
// were at b0 and written out as entries (key = table * n + row, a d-vector).  A stable
// LSD radix sort on the keys (4-bit digits, per-thread sequential ranking, so equal
// keys keep the order in which they were emitted: by sample, then order, then slot)
// groups the entries of each row; each row's entries are then summed left to right in
// binary32 and the sum is added to the row once.  No atomics touch the numbers, so the
// result is the same on every run.
#include "handle.hpp"
#include "scan.hpp"
#include "tile.hpp"
#include "sgd_kernels.hpp"

namespace lh {

LH_DECLARE_LAUNCHERS(float, 1)
LH_DECLARE_LAUNCHERS(float, 2)
LH_DECLARE_LAUNCHERS(float, 3)
LH_DECLARE_LAUNCHERS(uint16_t, 1)
LH_DECLARE_LAUNCHERS(uint16_t, 2)
LH_DECLARE_LAUNCHERS(uint16_t, 3)

// ---- radix sort -------------------------------------------------------------
__global__ void __launch_bounds__(RADIX_THREADS) k_radix_hist(const uint32_t *keys, long long E, int shift,
                                                              uint32_t *hist, long long nblk)
{
    __shared__ uint32_t cnt[16];
    if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
    __syncthreads();
    long long base = (long long)blockIdx.x * RADIX_TILE;
    for (int i = threadIdx.x; i < RADIX_TILE; i += RADIX_THREADS) {
        long long e = base + i;
        if (e < E) atomicAdd(&cnt[(keys[e] >> shift) & 15u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 16) hist[(long long)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// hist_incl: inclusive scan of hist in digit-major order.
__global__ void __launch_bounds__(RADIX_THREADS) k_radix_scatter(const uint32_t *kin, const uint32_t *vin,
                                                                 uint32_t *kout, uint32_t *vout, long long E,
                                                                 int shift, const uint32_t *hist_incl,
                                                                 long long nblk)
{
    __shared__ uint32_t cnt[16][RADIX_THREADS + 1];
    __shared__ uint32_t tot[16];
    const int t = threadIdx.x;
    const long long base = (long long)blockIdx.x * RADIX_TILE + (long long)t * RADIX_ITEMS;
#pragma unroll
    for (int dgt = 0; dgt < 16; ++dgt) cnt[dgt][t] = 0;
    for (int i = 0; i < RADIX_ITEMS; ++i) {
        long long e = base + i;
        if (e < E) cnt[(kin[e] >> shift) & 15u][t] += 1;
    }
    __syncthreads();
    if (t < 16) {  // exclusive scan over threads for digit t
        uint32_t run = 0;
        for (int j = 0; j < RADIX_THREADS; ++j) {
            uint32_t c = cnt[t][j];
            cnt[t][j] = run;
            run += c;
        }
        tot[t] = run;
    }
    __syncthreads();
    for (int i = 0; i < RADIX_ITEMS; ++i) {
        long long e = base + i;
        if (e < E) {
            uint32_t k = kin[e];
            uint32_t dgt = (k >> shift) & 15u;
            uint32_t start = hist_incl[(long long)dgt * nblk + blockIdx.x] - tot[dgt];
            uint32_t pos = start + cnt[dgt][t];
            cnt[dgt][t] += 1;
            kout[pos] = k;
            vout[pos] = vin[e];
        }
    }
}

void radix_sort_u32(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, long long E, int bits, uint32_t *hist,
                    uint32_t *ilev, hipStream_t s, uint32_t **kout, uint32_t **vout)
{
    const int passes = (bits + 3) / 4;
    const long long nblk = LH_CDIV(E, RADIX_TILE);
    for (int ps = 0; ps < passes && E > 0; ++ps) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(RADIX_THREADS), 0, s, ka, E, 4 * ps, hist, nblk);
        chunk_scan<OpAdd<uint32_t>>(hist, hist, 16 * nblk, ilev, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(RADIX_THREADS), 0, s, ka, va, kb, vb, E, 4 * ps,
                           hist, nblk);
        uint32_t *t = ka;
        ka = kb;
        kb = t;
        t = va;
        va = vb;
        vb = t;
    }
    *kout = ka;
    *vout = va;
}

// ---- segments ---------------------------------------------------------------
__global__ void k_heads(const uint32_t *keys, long long E, uint32_t *flag)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void k_seg_starts(const uint32_t *keys, const uint32_t *segid, long long E, uint32_t *start)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    if (i == 0 || keys[i] != keys[i - 1]) start[segid[i] - 1] = (uint32_t)i;
}

// One group of LPS lanes per touched row: sum its entries in order, add once.
template <typename TT, int LPS>
__global__ void __launch_bounds__(256) k_apply(GraphDev g, const uint32_t *keys, const uint32_t *vals,
                                               const uint32_t *start, const uint32_t *segid, long long E,
                                               const float *contrib, unsigned long long batch_idx)
{
    constexpr int EPU = Elem<TT>::EPU;
    constexpr int GPB = 256 / LPS;
    const long long nseg = E > 0 ? (long long)segid[E - 1] : 0;
    const int gl = threadIdx.x % LPS;
    const long long seg = (long long)blockIdx.x * GPB + threadIdx.x / LPS;
    if (seg >= nseg) return;
    const long long p0 = start[seg];
    const long long p1 = seg + 1 < nseg ? (long long)start[seg + 1] : E;
    const uint32_t key = keys[p0];
    const int table = (int)(key / (uint32_t)g.n);
    const long long row = (long long)(key % (uint32_t)g.n);
    uint32_t *X = reinterpret_cast<uint32_t *>((TT *)g.tab[table] + row * g.d);
    for (int un = gl; un < g.nunits; un += LPS) {
        float acc[EPU];
#pragma unroll
        for (int e = 0; e < EPU; ++e) acc[e] = 0.f;
        for (long long p = p0; p < p1; ++p) {
            const float *c = contrib + (unsigned long long)vals[p] * g.d + un * EPU;
#pragma unroll
            for (int e = 0; e < EPU; ++e) acc[e] += c[e];
        }
        float x[EPU];
        unit_to_f32<TT>(X[un], x);
#pragma unroll
        for (int e = 0; e < EPU; ++e) x[e] += acc[e];
        uint32_t rnd = 0u;
        if constexpr (EPU == 2) {
            // Stochastic rounding bits: Philox4x64-10 keyed by (batch, table, row); block
            // un / 8 holds 32 bits for each of 8 units.
            u64x4 r = philox4x64_10(g.seed, g.sr_key, batch_idx, (unsigned long long)table,
                                    (unsigned long long)row, (unsigned long long)(un / 8));
            const int q = (un % 8) / 2;
            unsigned long long wd = q == 0 ? r.x : q == 1 ? r.y : q == 2 ? r.z : r.w;
            rnd = (uint32_t)(wd >> (32 * (un % 2)));
        }
        X[un] = f32_to_unit<TT>(x, rnd);
    }
}

static hipError_t launch_contrib(const GraphDev &g, int dtype, int orders, const TileCfg &c,
                                 unsigned long long b0, unsigned long long b1, int num_cu, const SnapOut &so,
                                 hipStream_t s)
{
    if (dtype == LH_FP32) {
        if (orders == 1) return launch_snap_t<float, 1>(g, c, b0, b1, num_cu, so, s);
        if (orders == 2) return launch_snap_t<float, 2>(g, c, b0, b1, num_cu, so, s);
        return launch_snap_t<float, 3>(g, c, b0, b1, num_cu, so, s);
    }
    if (orders == 1) return launch_snap_t<uint16_t, 1>(g, c, b0, b1, num_cu, so, s);
    if (orders == 2) return launch_snap_t<uint16_t, 2>(g, c, b0, b1, num_cu, so, s);
    return launch_snap_t<uint16_t, 3>(g, c, b0, b1, num_cu, so, s);
}

lh_status train_snapshot(lh_handle *h, unsigned long long first, unsigned long long count, const int2 *pairs,
                         unsigned long long pairs_first)
{
    const lh_params &p = h->p;
    const WsLayout &L = h->lay;
    GraphDev g = graph_dev(h);
    g.pairs = pairs;
    g.pairs_first = pairs_first;
    g.pool_n = pairs ? h->walk.pool : 0;
    hipStream_t s = h->stream;
    const unsigned long long B = (unsigned long long)p.batch;
    const int nord = p.orders == 3 ? 2 : 1;
    const unsigned long long per = (unsigned long long)nord * (unsigned long long)(p.K + 2);
    uint32_t *k0 = (uint32_t *)(h->ws + L.keys0), *k1 = (uint32_t *)(h->ws + L.keys1);
    uint32_t *v0 = (uint32_t *)(h->ws + L.vals0), *v1 = (uint32_t *)(h->ws + L.vals1);
    float *contrib = (float *)(h->ws + L.contrib);
    uint32_t *hist = (uint32_t *)(h->ws + L.hist);
    uint32_t *ilev = (uint32_t *)(h->ws + L.ilev);
    uint32_t *seg = (uint32_t *)(h->ws + L.seg);
    uint32_t *segid = (uint32_t *)(h->ws + L.segid);
    // key bits: keys < 3n
    int bits = 1;
    while (bits < 32 && (1ull << bits) < 3ull * (unsigned long long)h->n) ++bits;
    TileCfg c = natural_cfg(p.dtype, p.d);
    const int apply_lps = c.lps;

    const unsigned long long end = first + count;
    for (unsigned long long b0 = first; b0 < end;) {
        unsigned long long b1 = (b0 / B + 1) * B;
        if (b1 > end) b1 = end;
        const long long E = (long long)((b1 - b0) * per);
        SnapOut so{k0, v0, contrib, b0, nord};
        hipError_t e = launch_contrib(g, p.dtype, p.orders, c, b0, b1, h->num_cu, so, s);
        if (e != hipSuccess) return hip_fail(h, e, "snapshot contributions");
        uint32_t *ka = k0, *va = v0;
        radix_sort_u32(k0, v0, k1, v1, E, bits, hist, ilev, s, &ka, &va);
        const unsigned eb = (unsigned)LH_CDIV(E, 256);
        hipLaunchKernelGGL(k_heads, dim3(eb), dim3(256), 0, s, ka, E, segid);
        chunk_scan<OpAdd<uint32_t>>(segid, segid, E, ilev, s);
        hipLaunchKernelGGL(k_seg_starts, dim3(eb), dim3(256), 0, s, ka, segid, E, seg);
        const unsigned ab = (unsigned)LH_CDIV(E, 256 / apply_lps);
        const unsigned long long bidx = b0 / B;
        if (p.dtype == LH_FP32) {
            switch (apply_lps) {
#define LH_AP(L)                                                                                                 \
    case L:                                                                                                      \
        hipLaunchKernelGGL((k_apply<float, L>), dim3(ab), dim3(256), 0, s, g, ka, va, seg, segid, E, contrib, bidx); \
        break;
                LH_AP(2) LH_AP(4) LH_AP(8) LH_AP(16) LH_AP(32) LH_AP(64)
#undef LH_AP
            }
        } else {
            switch (apply_lps) {
#define LH_AP(L)                                                                                                    \
    case L:                                                                                                         \
        hipLaunchKernelGGL((k_apply<uint16_t, L>), dim3(ab), dim3(256), 0, s, g, ka, va, seg, segid, E, contrib, bidx); \
        break;
                LH_AP(2) LH_AP(4) LH_AP(8) LH_AP(16) LH_AP(32) LH_AP(64)
#undef LH_AP
            }
        }
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(h, e, "snapshot apply");
        b0 = b1;
    }
    return LH_OK;
}

}  // namespace lh
