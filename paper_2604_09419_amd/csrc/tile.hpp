// The per-sample body of LINE edge-sampled SGD on gfx950, shared by the single-graph
// Hogwild kernels, the SNAPSHOT contribution kernel and the batched persistent kernel.
//
// One wavefront handles a tile of 64 consecutive sample indices:
//   phase A  lane l draws sample (tile + l): 1 + K Philox4x64-10 blocks, one 32-byte
//            edge record and K 16-byte negative records (Algorithm 3 root edge,
//            Eq. (1) negatives), plus a bit mask of repeated rows in the tuple;
//   phase B  groups of LPS lanes take the 64 samples in LPS rounds.  Each lane holds
//            CPL 16-byte chunks of every row (128-bit loads, a row's chunks spread over
//            the group so the group reads whole rows coalesced), the 1 + K dot products
//            are reduced across the group with cross-lane shuffles, and the updates of
//            Algorithm 1 / Eqs. (2)-(3) are written back (Hogwild: plain stores, no
//            locks) or emitted as per-row contributions (SNAPSHOT, Eq. (4)).
// All 1 + K dot products of a sample use the rows as loaded before the sample; a row
// that appears in several slots of one sample receives the sum of its increments.
#pragma once

#include "handle.hpp"

namespace lh {

template <typename TT>
struct Elem;
template <>
struct Elem<float> {
    static constexpr int VEC = 4;  // 16 bytes of binary32
};
template <>
struct Elem<uint16_t> {
    static constexpr int VEC = 8;  // 16 bytes of bfloat16
};

template <typename TT>
__device__ __forceinline__ void load_chunk(const TT *row, int ch, float (&o)[Elem<TT>::VEC]);

template <>
__device__ __forceinline__ void load_chunk<float>(const float *row, int ch, float (&o)[4])
{
    float4 v = *reinterpret_cast<const float4 *>(row + (size_t)ch * 4);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
}

template <>
__device__ __forceinline__ void load_chunk<uint16_t>(const uint16_t *row, int ch, float (&o)[8])
{
    uint4 v = *reinterpret_cast<const uint4 *>(row + (size_t)ch * 8);
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        o[2 * i] = __uint_as_float(w[i] << 16);
        o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
}

// Store one chunk.  bfloat16 rows use stochastic rounding with bits from lowbias32 of
// (sample seed + chunk counter); binary32 rows are stored as computed.
template <typename TT>
__device__ __forceinline__ void store_chunk(TT *row, int ch, const float (&x)[Elem<TT>::VEC],
                                            uint32_t sr, uint32_t ctr);

template <>
__device__ __forceinline__ void store_chunk<float>(float *row, int ch, const float (&x)[4], uint32_t,
                                                   uint32_t)
{
    *reinterpret_cast<float4 *>(row + (size_t)ch * 4) = make_float4(x[0], x[1], x[2], x[3]);
}

template <>
__device__ __forceinline__ void store_chunk<uint16_t>(uint16_t *row, int ch, const float (&x)[8],
                                                      uint32_t sr, uint32_t ctr)
{
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t r = lowbias32(sr + (ctr * 4u + (uint32_t)i) * 0x9E3779B9u);
        uint32_t lo = f32_to_bf16_sr(x[2 * i], r);
        uint32_t hi = f32_to_bf16_sr(x[2 * i + 1], r >> 16);
        w[i] = lo | (hi << 16);
    }
    *reinterpret_cast<uint4 *>(row + (size_t)ch * 8) = make_uint4(w[0], w[1], w[2], w[3]);
}

// Where SNAPSHOT contributions go.
struct SnapOut {
    uint32_t *keys;      // [entries]  table * n + row
    uint32_t *vals;      // [entries]  entry index
    float *contrib;      // [entries x d]
    unsigned long long base;  // first sample of the batch
    int nord;            // orders per sample (1 or 2)
};

// Sum over an aligned group of LPS lanes, every lane receiving the sum.  Within a row
// of 16 lanes the butterfly uses DPP: quad_perm [1,0,3,2] and [2,3,0,1] (xor 1, 2), then
// row_half_mirror and row_mirror, which pair each lane with a lane of the other half
// once the halves are uniform.  Across rows: ds_swizzle xor 16, then a shuffle xor 32.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, true));
}

template <int LPS>
__device__ __forceinline__ float group_sum(float x)
{
    if constexpr (LPS >= 2) x += dpp_mov<0xB1>(x);   // quad_perm [1,0,3,2]
    if constexpr (LPS >= 4) x += dpp_mov<0x4E>(x);   // quad_perm [2,3,0,1]
    if constexpr (LPS >= 8) x += dpp_mov<0x141>(x);  // row_half_mirror
    if constexpr (LPS >= 16) x += dpp_mov<0x140>(x); // row_mirror
    if constexpr (LPS >= 32)
        x += __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x), 0x401F));
    if constexpr (LPS >= 64) x += __shfl_xor(x, 32);
    return x;
}

// This lane's chunks of the 2 + K rows of one order of one sample, as loaded.
template <typename TT, int CPL, int KMAX>
struct Rows {
    float a[CPL][Elem<TT>::VEC];
    float b[KMAX + 1][CPL][Elem<TT>::VEC];
};

template <typename TT, int LPS, int CPL, int KMAX>
__device__ __forceinline__ void load_rows(Rows<TT, CPL, KMAX> &r, const GraphDev &g, const TT *A, const TT *B,
                                          int u, const int (&ids)[KMAX + 1], int K, int gl)
{
    constexpr int VEC = Elem<TT>::VEC;
    const int d = g.d, nch = g.nch;
    const TT *arow = A + (long long)u * d;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        int ch = c * LPS + gl;
        if (ch < nch) {
            load_chunk<TT>(arow, ch, r.a[c]);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) r.a[c][e] = 0.f;
        }
    }
#pragma unroll
    for (int j = 0; j <= KMAX; ++j) {
        const TT *brow = B + (long long)ids[j] * d;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            int ch = c * LPS + gl;
            if (j <= K && ch < nch) {
                load_chunk<TT>(brow, ch, r.b[j][c]);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) r.b[j][c][e] = 0.f;
            }
        }
    }
}

// One order of one sample, rows already loaded.  A holds the vertex rows, B the context
// rows (A == B for first order).  ids[0] = v, ids[1..K] = negatives.
template <typename TT, int LPS, int CPL, int KMAX, bool FIRST, bool SNAP>
__device__ __forceinline__ void sgd_order(const GraphDev &g, TT *A, TT *B, int u, const int (&ids)[KMAX + 1],
                                          int K, float eta, unsigned dupb, unsigned dupu, uint32_t sr,
                                          int oi, int gl, const SnapOut &so, unsigned long long s,
                                          int tabA, int tabB, const Rows<TT, CPL, KMAX> &rows)
{
    constexpr int VEC = Elem<TT>::VEC;
    const int d = g.d, nch = g.nch;
    const auto &a = rows.a;
    const auto &b = rows.b;
    float gj[KMAX + 1];
#pragma unroll
    for (int j = 0; j <= KMAX; ++j) {
        float x = 0.f;
#pragma unroll
        for (int c = 0; c < CPL; ++c)
#pragma unroll
            for (int e = 0; e < VEC; ++e) x = fmaf(a[c][e], b[j][c][e], x);
        gj[j] = x;
    }
#pragma unroll
    for (int j = 0; j <= KMAX; ++j) gj[j] = group_sum<LPS>(gj[j]);
#pragma unroll
    for (int j = 0; j <= KMAX; ++j) {
        float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-gj[j]));
        float gg = j == 0 ? eta * (1.0f - sg) : -eta * g.alpha * sg;
        gj[j] = j <= K ? gg : 0.f;
    }
    const float el = eta * g.lambda;

    // dA = sum_j g_j b_j - (1 + K) eta lambda a
    float dA[CPL][VEC];
    const float decayA = (float)(K + 1) * el;
#pragma unroll
    for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            float acc = -decayA * a[c][e];
#pragma unroll
            for (int j = 0; j <= KMAX; ++j) acc = fmaf(gj[j], b[j][c][e], acc);
            dA[c][e] = acc;
        }

    if constexpr (SNAP) {
        // Entries of this sample/order: slot 0 = A[u] (dA), slot 1 + j = B[ids[j]] (delta_j).
        const unsigned long long e0 =
            ((s - so.base) * (unsigned long long)so.nord + (unsigned long long)oi) * (unsigned long long)(K + 2);
        float *crow = so.contrib + e0 * (unsigned long long)d;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            int ch = c * LPS + gl;
            if (ch < nch) {
                float *p = crow + ch * 4 * (VEC / 4);
#pragma unroll
                for (int q = 0; q < VEC / 4; ++q)
                    *reinterpret_cast<float4 *>(p + 4 * q) =
                        make_float4(dA[c][4 * q], dA[c][4 * q + 1], dA[c][4 * q + 2], dA[c][4 * q + 3]);
            }
        }
#pragma unroll
        for (int j = 0; j <= KMAX; ++j) {
            if (j > K) break;
            float *brow = crow + (unsigned long long)(j + 1) * d;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                int ch = c * LPS + gl;
                if (ch < nch) {
                    float t[VEC];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) t[e] = gj[j] * a[c][e] - el * b[j][c][e];
                    float *p = brow + ch * VEC;
#pragma unroll
                    for (int q = 0; q < VEC / 4; ++q)
                        *reinterpret_cast<float4 *>(p + 4 * q) =
                            make_float4(t[4 * q], t[4 * q + 1], t[4 * q + 2], t[4 * q + 3]);
                }
            }
        }
        if (gl == 0) {
            so.keys[e0] = (uint32_t)((long long)tabA * g.n + u);
            so.vals[e0] = (uint32_t)e0;
#pragma unroll
            for (int j = 0; j <= KMAX; ++j) {
                if (j > K) break;
                so.keys[e0 + 1 + j] = (uint32_t)((long long)tabB * g.n + ids[j]);
                so.vals[e0 + 1 + j] = (uint32_t)(e0 + 1 + j);
            }
        }
        return;
    } else {
        // Merge repeated rows: slot j's total step is Gm[j] (sum of the g of all slots
        // with that row) and cm[j] (their number, for the decay); slots that repeat an
        // earlier row (or, in first order, the vertex row u) store nothing.
        float Gm[KMAX + 1], cm[KMAX + 1];
        float GA = 0.f, cA = 0.f;
        unsigned skip = 0;
#pragma unroll
        for (int j = 0; j <= KMAX; ++j) {
            Gm[j] = gj[j];
            cm[j] = j <= K ? 1.f : 0.f;
        }
        if (dupb | (FIRST ? dupu : 0u)) {
#pragma unroll
            for (int j = 0; j <= KMAX; ++j) {
                if (j > K) break;
                if (FIRST && ids[j] == u) {
                    GA += gj[j];
                    cA += 1.f;
                    Gm[j] = 0.f;
                    cm[j] = 0.f;
                    skip |= 1u << j;
                    continue;
                }
                int own = j;
#pragma unroll
                for (int jj = KMAX; jj >= 0; --jj)
                    if (jj < j && ids[jj] == ids[j]) own = jj;
                if (own != j) {
#pragma unroll
                    for (int jj = 0; jj <= KMAX; ++jj)
                        if (jj == own) {
                            Gm[jj] += gj[j];
                            cm[jj] += 1.f;
                        }
                    Gm[j] = 0.f;
                    cm[j] = 0.f;
                    skip |= 1u << j;
                }
            }
        }
        // vertex row
        TT *wa = A + (long long)u * d;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            int ch = c * LPS + gl;
            if (ch < nch) {
                float o[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    float t = a[c][e] + dA[c][e];
                    if (FIRST) t += GA * a[c][e] - cA * el * a[c][e];
                    o[e] = t;
                }
                store_chunk<TT>(wa, ch, o, sr, (uint32_t)((oi * (KMAX + 2)) * 64 + ch));
            }
        }
        // context rows
#pragma unroll
        for (int j = 0; j <= KMAX; ++j) {
            if (j > K) break;
            if (skip & (1u << j)) continue;
            TT *wb = B + (long long)ids[j] * d;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                int ch = c * LPS + gl;
                if (ch < nch) {
                    float o[VEC];
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        o[e] = b[j][c][e] + (Gm[j] * a[c][e] - cm[j] * el * b[j][c][e]);
                    store_chunk<TT>(wb, ch, o, sr, (uint32_t)((oi * (KMAX + 2) + 1 + j) * 64 + ch));
                }
            }
        }
    }
}

// One tile of 64 samples [tile, min(tile + 64, end)).
template <typename TT, int LPS, int CPL, int KMAX, int ORD, bool SNAP>
__device__ __forceinline__ void sgd_tile(const GraphDev &g, unsigned long long tile, unsigned long long end,
                                         const SnapOut &so)
{
    static_assert(LPS >= 1 && LPS <= 64 && (64 % LPS) == 0, "lanes per sample divide the wavefront");
    constexpr int GPW = 64 / LPS;
    const int lane = threadIdx.x & 63;
    const int grp = lane / LPS, gl = lane % LPS;
    const int K = g.K;

    // ---- phase A: one lane per sample --------------------------------------
    int my_u = 0, my_ids[KMAX + 1];
    unsigned my_dup = 0;
    uint32_t my_sr = 0;
    float my_eta = 0.f;
#pragma unroll
    for (int j = 0; j <= KMAX; ++j) my_ids[j] = 0;
    {
        const unsigned long long s = tile + (unsigned long long)lane;
        if (s < end) {
            // One Philox block at a time, its record load issued at once, so the loads of
            // all 1 + K slots are in flight together while the blocks are not interleaved
            // (which would hold 1 + K blocks of state in registers).
            u64x4 x0 = philox4x64_10(g.seed, g.key1, s, 0ull, 0ull, 0ull);
            long long ce = draw_column(x0.x, g.m);
            const uint4 *er = reinterpret_cast<const uint4 *>(g.erec + ce);
            uint4 r0 = er[0], r1 = er[1];
            const unsigned long long x0y = x0.y;
            my_sr = (uint32_t)x0.z;
            __builtin_amdgcn_sched_barrier(0);
            unsigned long long xy[KMAX];
            int cn[KMAX];
            uint4 nr[KMAX];
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < K) {
                    u64x4 x = philox4x64_10(g.seed, g.key1, s, (unsigned long long)(j + 1), 0ull, 0ull);
                    cn[j] = (int)draw_column(x.x, g.n);
                    xy[j] = x.y;
                    nr[j] = *reinterpret_cast<const uint4 *>(g.nrec + cn[j]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            my_eta = (float)(g.eta0 * (1.0 - (double)s / (double)g.T)) * g.eta_scale;
            unsigned long long ethr = (unsigned long long)r0.x | ((unsigned long long)r0.y << 32);
            bool keep = x0y < ethr;
            my_u = keep ? (int)r0.w : (int)r1.y;
            my_ids[0] = keep ? (int)r1.x : (int)r1.z;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < K) {
                    unsigned long long nthr = (unsigned long long)nr[j].x | ((unsigned long long)nr[j].y << 32);
                    my_ids[j + 1] = xy[j] < nthr ? cn[j] : (int)nr[j].z;
                }
            }
            // repeated rows among (v, n_1..n_K) in the low half, rows equal to u in the high half
#pragma unroll
            for (int j = 0; j <= KMAX; ++j) {
                if (j > K) break;
                if (my_ids[j] == my_u) my_dup |= 1u << (16 + j);
#pragma unroll
                for (int jj = 0; jj < j; ++jj)
                    if (my_ids[jj] == my_ids[j]) my_dup |= 1u << j;
            }
        }
    }

    // ---- phase B: LPS lanes per sample ----------------------------------------
    for (int r = 0; r < LPS; ++r) {
        const int src = r * GPW + grp;
        const int u = __shfl(my_u, src);
        int ids[KMAX + 1];
#pragma unroll
        for (int j = 0; j <= KMAX; ++j) ids[j] = __shfl(my_ids[j], src);
        const unsigned dup = (unsigned)__shfl((int)my_dup, src);
        uint32_t sr = 0;
        if constexpr (sizeof(TT) == 2 && !SNAP) sr = (uint32_t)__shfl((int)my_sr, src);
        const float eta = __shfl(my_eta, src);  // every cross-lane read before lanes diverge
        const unsigned long long s = tile + (unsigned long long)src;
        if (s >= end) continue;
        const unsigned dupb = dup & 0xffffu, dupu = dup >> 16;
        // Issue the row loads of both orders before any arithmetic or store, so that up to
        // 2 (2 + K) rows per sample are in flight at once.
        Rows<TT, CPL, KMAX> r2, r1;
        if constexpr ((ORD & 2) != 0)
            load_rows<TT, LPS, CPL, KMAX>(r2, g, (const TT *)g.tab[0], (const TT *)g.tab[1], u, ids, K, gl);
        if constexpr ((ORD & 1) != 0)
            load_rows<TT, LPS, CPL, KMAX>(r1, g, (const TT *)g.tab[2], (const TT *)g.tab[2], u, ids, K, gl);
        int oi = 0;
        if constexpr ((ORD & 2) != 0) {
            sgd_order<TT, LPS, CPL, KMAX, false, SNAP>(g, (TT *)g.tab[0], (TT *)g.tab[1], u, ids, K, eta, dupb,
                                                       dupu, sr, oi, gl, so, s, LH_TABLE_U, LH_TABLE_C, r2);
            ++oi;
        }
        if constexpr ((ORD & 1) != 0) {
            sgd_order<TT, LPS, CPL, KMAX, true, SNAP>(g, (TT *)g.tab[2], (TT *)g.tab[2], u, ids, K, eta, dupb,
                                                      dupu, sr ^ 0x5bd1e995u, oi, gl, so, s, LH_TABLE_U1,
                                                      LH_TABLE_U1, r1);
        }
    }
}

}  // namespace lh
