// The per-sample body of LINE edge-sampled SGD on gfx950, shared by the single-graph
// Hogwild kernels, the SNAPSHOT contribution kernel and the batched persistent kernel.
//
// One wavefront handles a tile of 64 consecutive sample indices:
//   phase A  lane l draws sample (tile + l): 1 + K Philox4x64-10 blocks, one 32-byte
//            edge record and K 16-byte negative records (Algorithm 3 root edge,
//            Eq. (1) negatives), a bit mask of rows repeated inside the tuple and a bit
//            mask of hot rows, and the sample's step size;
//   phase B  groups of LPS lanes take the 64 samples in LPS rounds.  A row is a run of
//            4-byte units (one binary32 value, or two bfloat16 values); lane gl of a
//            group holds units gl, gl + LPS, gl + 2 LPS, ... so every load, store and
//            atomic instruction of the group covers LPS consecutive units.  The 1 + K
//            dot products are reduced across the group with DPP, and the updates of
//            Algorithm 1 / Eqs. (2)-(3) are written back (HOGWILD) or emitted as
//            per-row contributions (SNAPSHOT, Eq. (4)).
//
// HOGWILD write-back: a cold row is stored (row as loaded plus the sample's increment;
// no locks) with a system-scope store (binary32 rows of a one-sample wavefront: a
// system-scope non-temporal buffer store), and every table row is loaded with system scope,
// so the eight XCDs' L2 caches never hold diverging copies.  A hot row -- one that an
// in-flight sample is likely to share, a hub -- is updated with atomic increments so that
// concurrent updates are not lost: binary32 atomics for binary32 tables; for bfloat16
// tables packed bfloat16 atomics of the increment rounded stochastically onto the row's
// bfloat16 grid, or (on request) binary32 atomics into a binary32 shadow of the hot rows
// that is rounded back into the table after the launch.
//
// All 1 + K dot products of a sample use the rows as loaded before the sample; a row
// that appears in several slots of one sample receives the sum of its increments (each
// occurrence is applied atomically).
#pragma once

#include "handle.hpp"

namespace lh {

template <typename TT>
struct Elem;
template <>
struct Elem<float> {
    static constexpr int EPU = 1;  // elements per 4-byte unit
};
template <>
struct Elem<uint16_t> {
    static constexpr int EPU = 2;
};

// ---- one 4-byte unit ----------------------------------------------------------------
template <typename TT>
__device__ __forceinline__ void unit_to_f32(uint32_t w, float (&o)[Elem<TT>::EPU])
{
    if constexpr (sizeof(TT) == 4) {
        o[0] = __uint_as_float(w);
    } else {
        o[0] = __uint_as_float(w << 16);
        o[1] = __uint_as_float(w & 0xffff0000u);
    }
}

// Pack a unit's values; bfloat16 with stochastic rounding from 32 random bits.
template <typename TT>
__device__ __forceinline__ uint32_t f32_to_unit(const float (&x)[Elem<TT>::EPU], uint32_t rnd)
{
    if constexpr (sizeof(TT) == 4) {
        return __float_as_uint(x[0]);
    } else {
        return bf16x2_sr(x[0], x[1], rnd);
    }
}

// ---- drawing one sample (shared by the parity hook k_sample and phase A) ------------
// Slot j of sample s (0: the positive arc, Algorithm 3's root edge; 1..K: negatives of
// Eq. (1), Algorithm 1) uses Philox4x64-10 block (key (seed, graph_id), counter
// (s, j, 0, 0)): column floor(x0 N / 2^64), kept when x1 < thr[column], else its alias.
struct SlotDraw {
    long long col;             // column of the alias table
    unsigned long long x1;     // threshold word
    unsigned long long x2;     // a spare word of the block (seeds of the rounding bits)
};

__device__ __forceinline__ SlotDraw draw_slot(const GraphDev &g, unsigned long long s, int j, long long N)
{
    const u64x4 x = philox4x64_10(g.seed, g.key1, s, (unsigned long long)j, 0ull, 0ull);
    return SlotDraw{draw_column(x.x, N), x.y, x.z};
}

// The 32-byte edge record of a column as two 16-byte words (one sector).  NT: loaded with
// the non-temporal hint.  Columns are uniform over the arcs, so an edge record is almost
// never read twice while cached; with bfloat16 tables the hint leaves the caches to rows
// and negative records (C3: 293.8 against 302.4-304.4 ms).  With binary32 tables it
// measured 0.2 % slower, so those keep the plain load.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

template <bool NT = false>
__device__ __forceinline__ void load_edge_rec(const EdgeRec *erec, long long col, uint4 &r0, uint4 &r1)
{
    if constexpr (NT) {
        const u32x4_t *er = reinterpret_cast<const u32x4_t *>(erec + col);
        const u32x4_t a = __builtin_nontemporal_load(er), b = __builtin_nontemporal_load(er + 1);
        r0 = make_uint4(a.x, a.y, a.z, a.w);
        r1 = make_uint4(b.x, b.y, b.z, b.w);
    } else {
        const uint4 *er = reinterpret_cast<const uint4 *>(erec + col);
        r0 = er[0];
        r1 = er[1];
    }
}

// Columns of slot 0's draw: the edge table's arcs, or the pair pool's collected pairs.
__device__ __forceinline__ long long slot0_columns(const GraphDev &g)
{
    return g.pool_n ? (long long)g.pool_n : g.m;
}

// Slot 0's record words: the edge table's record of the drawn column (Algorithm 3's root
// edge), or, when the positive pairs come from random walks, a record that yields the
// sample's walk pair (u, v) whatever the threshold word (both outcomes are (u, v)), with
// the heats of u and v in the record's heat word.  With a pair pool (Sec. IV-C,
// Augmented-Pair) the pair is the first vertex of collected pair col (the first column
// draw) and the second vertex of collected pair floor(x1 R / 2^64) (the second word).
template <bool NT = false>
__device__ __forceinline__ void load_pair_rec(const GraphDev &g, unsigned long long s, long long col,
                                              unsigned long long x1, uint4 &r0, uint4 &r1)
{
    if (g.pairs == nullptr) {
        load_edge_rec<NT>(g.erec, col, r0, r1);
        return;
    }
    int2 p;
    if (g.pool_n) {
        p.x = g.pairs[col].x;
        p.y = g.pairs[draw_column(x1, (long long)g.pool_n)].y;
    } else {
        p = g.pairs[s - g.pairs_first];
    }
    const unsigned hu = g.heat[p.x], hv = g.heat[p.y];
    r0 = make_uint4(~0u, ~0u, 0u, (unsigned)p.x);
    r1 = make_uint4((unsigned)p.y, (unsigned)p.x, (unsigned)p.y, hu | (hv << 8) | (hu << 16) | (hv << 24));
}

// The arc (u, v) a slot-0 draw picks from its record words (threshold r0.xy, column arc's
// endpoints r0.w, r1.x, alias arc's r1.y, r1.z); returns whether the column kept itself.
__device__ __forceinline__ bool edge_pick(const uint4 &r0, const uint4 &r1, unsigned long long x1, int &u, int &v)
{
    const unsigned long long thr = (unsigned long long)r0.x | ((unsigned long long)r0.y << 32);
    const bool keep = x1 < thr;
    u = keep ? (int)r0.w : (int)r1.y;
    v = keep ? (int)r1.x : (int)r1.z;
    return keep;
}

// The node a negative draw picks from its 16-byte record (threshold nr.xy, alias nr.z).
__device__ __forceinline__ bool neg_pick(const uint4 &nr, const SlotDraw &d, int &id)
{
    const unsigned long long thr = (unsigned long long)nr.x | ((unsigned long long)nr.y << 32);
    const bool keep = d.x1 < thr;
    id = keep ? (int)d.col : (int)nr.z;
    return keep;
}

// Where SNAPSHOT contributions go.
struct SnapOut {
    uint32_t *keys;           // [entries]  table * n + row
    uint32_t *vals;           // [entries]  entry index
    float *contrib;           // [entries x d], binary32
    unsigned long long base;  // first sample of the batch
    int nord;                 // orders per sample (1 or 2)
};

// Sum over an aligned group of LPS lanes, every lane receiving the sum.  Within a row
// of 16 lanes the butterfly uses DPP: quad_perm [1,0,3,2] and [2,3,0,1] (xor 1, 2), then
// row_half_mirror and row_mirror, which pair each lane with a lane of the other half
// once the halves are uniform.  Across rows, gfx950's lane swaps (v_permlane16_swap: rows
// 0 <-> 1 and 2 <-> 3; v_permlane32_swap: the two halves of the wavefront) give each
// lane its partner's value in one VALU instruction, with no LDS round trip.
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
    if constexpr (LPS >= 32) {
        // swapping a register with itself leaves the partner row's value in one of the two
        // results and this lane's own value in the other, so their sum is the pair's sum
        const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
        x = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    }
    if constexpr (LPS >= 64) {
        const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
        x = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    }
    return x;
}

// Phase B's read of a sample's value from the phase-A lane src that drew it: with one sample
// per wavefront src is uniform and the value is read into a scalar register (the sample's
// row addresses are then computed by the scalar unit); otherwise a cross-lane permute.
template <int LPS>
__device__ __forceinline__ int sample_lane(int v, int src)
{
    if constexpr (LPS == 64) return __builtin_amdgcn_readlane(v, src);
    else return __shfl(v, src);
}

// Lane j's value of this lane's group of LPS lanes (j < LPS): a scalar read when the group
// is the whole wavefront, a cross-lane permute otherwise.
template <int LPS>
__device__ __forceinline__ float group_lane(float x, int j)
{
    if constexpr (LPS == 64) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
    } else {
        const int base = (int)(threadIdx.x & 63u) & ~(LPS - 1);
        return __shfl(x, base + j);
    }
}

typedef short short2_t __attribute__((ext_vector_type(2)));

// Element e of a unit as binary32.
template <typename TT>
__device__ __forceinline__ float val(uint32_t w, int e)
{
    if constexpr (sizeof(TT) == 4) return __uint_as_float(w);
    return e == 0 ? __uint_as_float(w << 16) : __uint_as_float(w & 0xffff0000u);
}

// This lane's units of the 2 + K rows of one order of one sample, as loaded (raw words,
// widened where used, so bfloat16 rows take half the registers).
template <typename TT, int UPL, int KMAX>
struct Rows {
    uint32_t a[UPL];
    uint32_t b[KMAX + 1][UPL];
};

// Table rows are read and (when cold) written with system-scope accesses (sc0 sc1 on
// gfx950).  The eight XCDs' L2 caches are not kept coherent with each other for ordinary
// accesses: a row written by one XCD would stay dirty in that L2 while the others read
// the old copy from memory.  System scope makes the accesses coherent across XCDs, at
// about 1 % of the training kernel's speed (measured on the C2 workload).
__device__ __forceinline__ uint32_t load_coherent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void store_coherent(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// A cold binary32 row written by a whole wavefront (64 lanes per sample, so the row address
// is uniform): buffer stores through a descriptor of the row, with the system-scope bits and
// the non-temporal hint (cache policy sc0 | nt | sc1).  Measured on the C2 workload the
// training launch takes 539.9 instead of 568.8 ms at 2 workgroups per CU, and 520 ms at the
// 4 the tuner then picks; the same stores slow bfloat16 rows down (C3: 319.4 against
// 303.0 ms), so those keep the global store.  The descriptor's range is the row, so no store
// can leave it; its last word (0x00020000) is the 32-bit data format that untyped buffer
// accesses use on gfx9-family devices.
constexpr int kCpolSysNT = 1 | 2 | 16;
constexpr int kRawBufferWord3 = 0x00020000;

template <int LPS, int UPL, bool FULL>
__device__ __forceinline__ void store_row_stream(uint32_t *row, int nunits, int gl, const uint32_t (&word)[UPL])
{
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, (short)0, nunits * 4, kRawBufferWord3);
#pragma unroll
    for (int k = 0; k < UPL; ++k) {
        const int un = k * LPS + gl;
        if (FULL || un < nunits) __builtin_amdgcn_raw_buffer_store_b32(word[k], rs, un * 4, 0, kCpolSysNT);
    }
}

// FULL: the shape covers the row exactly (LPS * UPL == units per row) and the sample has
// exactly KMAX negatives, so no access needs a bounds mask or a slot test and the loads and
// stores of a sample are straight-line code.
template <typename TT, int LPS, int UPL, bool FULL>
__device__ __forceinline__ void load_row(const TT *row, int nunits, int gl, uint32_t (&o)[UPL])
{
    const uint32_t *w = reinterpret_cast<const uint32_t *>(row);
#pragma unroll
    for (int k = 0; k < UPL; ++k) {
        const int un = k * LPS + gl;
        uint32_t v = 0u;
        if (FULL || un < nunits) v = load_coherent(w + un);
        o[k] = v;
    }
}

// Raw words of row `id` of table t for this lane.  binary32: the row's units.  bfloat16:
// lo = the table row's units (two values each), or (id < 0) the even half of shadow row
// ~id as binary32 bits, with hi = its odd half (a shadow row holds the even elements of
// the row and then the odd ones, element 2 un + e at e * d / 2 + un, so the lanes of a
// group touch contiguous words for each half).  The address is chosen without a branch
// and nothing here uses the loaded words, so every row's loads of a sample are in flight
// together; shadow rows are packed afterwards by pack_shadow_row.  SH: the kernel may meet
// shadow rows (else ids are never negative and hi stays untouched).
template <typename TT, int LPS, int UPL, bool SH, bool FULL>
__device__ __forceinline__ void load_row_raw(const GraphDev &g, int t, int id, int gl, uint32_t (&lo)[UPL],
                                             uint32_t (&hi)[UPL])
{
    const int nu = g.nunits;
    if constexpr (sizeof(TT) == 4 || !SH) {
        load_row<TT, LPS, UPL, FULL>((const TT *)g.tab[t] + (long long)id * g.d, nu, gl, lo);
    } else {
        const bool sh = id < 0;
        const uint32_t *tw = reinterpret_cast<const uint32_t *>((const TT *)g.tab[t] + (long long)(sh ? 0 : id) * g.d);
        const uint32_t *sw = reinterpret_cast<const uint32_t *>(g.shadow[t] + (long long)(sh ? ~id : 0) * g.d);
        const uint32_t *pa = sh ? sw : tw;
#pragma unroll
        for (int k = 0; k < UPL; ++k) {
            const int un = k * LPS + gl;
            lo[k] = un < nu ? load_coherent(pa + un) : 0u;
            hi[k] = (sh && un < nu) ? load_coherent(sw + nu + un) : 0u;
        }
    }
}

// bfloat16: a shadow row's words become units rounded to nearest even (no-op otherwise).
template <typename TT, int UPL, bool SH>
__device__ __forceinline__ void pack_shadow_row(int id, uint32_t (&lo)[UPL], const uint32_t (&hi)[UPL])
{
    if constexpr (sizeof(TT) == 2 && SH) {
#pragma unroll
        for (int k = 0; k < UPL; ++k) {
            const uint32_t p = bf16x2_rne(__uint_as_float(lo[k]), __uint_as_float(hi[k]));
            lo[k] = id < 0 ? p : lo[k];
        }
    }
}

template <typename TT, int LPS, int UPL, int KMAX, bool SH, bool FULL>
__device__ __forceinline__ void load_rows(Rows<TT, UPL, KMAX> &r, const GraphDev &g, int tA, int tB, int u,
                                          const int (&ids)[KMAX + 1], int K, int gl)
{
    uint32_t ah[UPL], bh[KMAX + 1][UPL];
    load_row_raw<TT, LPS, UPL, SH, FULL>(g, tA, u, gl, r.a, ah);
#pragma unroll
    for (int j = 0; j <= KMAX; ++j) {
        if (FULL || j <= K) {
            load_row_raw<TT, LPS, UPL, SH, FULL>(g, tB, ids[j], gl, r.b[j], bh[j]);
        } else {
#pragma unroll
            for (int k = 0; k < UPL; ++k) r.b[j][k] = bh[j][k] = 0u;
        }
    }
    pack_shadow_row<TT, UPL, SH>(u, r.a, ah);
#pragma unroll
    for (int j = 0; j <= KMAX; ++j)
        if (FULL || j <= K) pack_shadow_row<TT, UPL, SH>(ids[j], r.b[j], bh[j]);
}

// Stochastic-rounding bits of unit un of a row: a Weyl step from the row's seed, one
// integer add once the lane's multiple of the step is formed.  Element 0 of the unit
// rounds with the low 16 bits, element 1 with the high 16 bits.  The row seeds of a
// sample come from one lowbias32 hash per sample and order (sgd_order), so each half is
// uniformly distributed and every rounding is unbiased.  The bits depend on the unit, not
// on the lane holding it, so every tile shape rounds alike.
__device__ __forceinline__ uint32_t sr_bits(uint32_t rseed, int un)
{
    return rseed + (uint32_t)un * 0x9E3779B9u;
}

// Write one row back: new = old + inc.  `hot` asks for the atomic path.
//   binary32: stored, or atomic increments;
//   bfloat16 table rows (id >= 0): with the random bits of unit un being rseed + un * phi
//   (element 0 rounds with its low half, element 1 with its high half), a cold row is
//   stored as the stochastic rounding SR(old + inc); a hot row receives, by packed bfloat16
//   atomic adds, the increments SR(old + inc) - old rounded to nearest (units whose
//   increments are both zero are skipped, except in a dry run).  While old and
//   SR(old + inc) are within a factor of two of each other (always when |inc| <= |old| / 2)
//   that difference is exact, and where no other write changed the unit since it was
//   loaded the atomic result is SR(old + inc) bit for bit, the value a cold store would have
//   written; near zero it may be one bfloat16 spacing off.  A concurrent change receives the
//   increment on top.  Shadow rows (id < 0, even elements then odd ones) get binary32
//   atomic increments.
template <typename TT, int LPS, int UPL, bool SH, bool FULL>
__device__ __forceinline__ void write_row(const GraphDev &g, int t, int id, int gl, const uint32_t (&old)[UPL],
                                          const float (&inc)[UPL][Elem<TT>::EPU], bool hot, uint32_t rseed)
{
    constexpr int EPU = Elem<TT>::EPU;
    const int nunits = g.nunits;
    if constexpr (EPU == 2 && SH) {
        if (id < 0) {
            float *sw = g.shadow[t] + (long long)(~id) * g.d;
#pragma unroll
            for (int k = 0; k < UPL; ++k) {
                const int un = k * LPS + gl;
                if (FULL || un < nunits) atomicAdd(sw + un, inc[k][0]);
            }
#pragma unroll
            for (int k = 0; k < UPL; ++k) {
                const int un = k * LPS + gl;
                if (FULL || un < nunits) atomicAdd(sw + nunits + un, inc[k][1]);
            }
            return;
        }
    }
    // The word of each unit, computed without branches: the new value (binary32), or its
    // stochastic rounding (bfloat16), for a store; the increment (binary32), or
    // SR(old + inc) - old rounded to nearest (bfloat16), for an atomic.  Then exactly one
    // memory instruction per unit, a store or an atomic.
    uint32_t word[UPL];
#pragma unroll
    for (int k = 0; k < UPL; ++k) {
        const int un = k * LPS + gl;
        if constexpr (EPU == 2) {
            const float o0 = val<TT>(old[k], 0), o1 = val<TT>(old[k], 1);
            const uint32_t nv = bf16x2_sr(o0 + inc[k][0], o1 + inc[k][1], sr_bits(rseed, un));
            const uint32_t p = bf16x2_rne(val<TT>(nv, 0) - o0, val<TT>(nv, 1) - o1);
            word[k] = hot ? p : nv;
        } else {
            const float o = val<TT>(old[k], 0);
            word[k] = __float_as_uint(hot ? inc[k][0] : o + inc[k][0]);
        }
    }
    uint32_t *w = reinterpret_cast<uint32_t *>((TT *)g.tab[t] + (long long)id * g.d);
    // Units whose bfloat16 increments are both zero are skipped, except in a dry run (step
    // size scaled to zero), so that a timing run pays for the hot set as training does, and
    // in FULL kernels, whose rows each take exactly one memory instruction per unit so that
    // the count of memory operations after each load is known to the compiler.
    const bool all = FULL || g.eta_scale == 0.0f;
    if (hot) {
#pragma unroll
        for (int k = 0; k < UPL; ++k) {
            const int un = k * LPS + gl;
            if (FULL || un < nunits) {
                if constexpr (EPU == 2) {
                    if (all || (word[k] & 0x7fff7fffu) != 0u)
                        __builtin_amdgcn_global_atomic_fadd_v2bf16(
                            (short2_t __attribute__((address_space(1))) *)(w + un),
                            __builtin_bit_cast(short2_t, word[k]));
                } else {
                    atomicAdd(reinterpret_cast<float *>(w) + un, __uint_as_float(word[k]));
                }
            }
        }
    } else if constexpr (LPS == 64 && sizeof(TT) == 4) {
        store_row_stream<LPS, UPL, FULL>(w, nunits, gl, word);
    } else {
#pragma unroll
        for (int k = 0; k < UPL; ++k) {
            const int un = k * LPS + gl;
            if (FULL || un < nunits) store_coherent(w + un, word[k]);
        }
    }
}

// One order of one sample, rows already loaded.  Table tabA holds the vertex rows, tabB
// the context rows (the same table for first order).  ids[0] = v, ids[1..K] = negatives
// (bfloat16 Hogwild: ~slot for rows in the shadow).  hot: bit 0 for the vertex row,
// bit 1 + j for slot j.
template <typename TT, int LPS, int UPL, int KMAX, bool FIRST, bool SNAP, bool SH, bool FULL>
__device__ __forceinline__ void sgd_order(const GraphDev &g, int u, const int (&ids)[KMAX + 1], int K, float eta,
                                          unsigned dupb, unsigned dupu, unsigned hot, uint32_t sr, int oi, int gl,
                                          const SnapOut &so, unsigned long long s, int tabA, int tabB,
                                          const Rows<TT, UPL, KMAX> &rows)
{
    constexpr int EPU = Elem<TT>::EPU;
    const int d = g.d, nu = g.nunits;
    const auto &a = rows.a;
    const auto &b = rows.b;
    float gj[KMAX + 1];
#pragma unroll
    for (int j = 0; j <= KMAX; ++j) {
        float x = 0.f;
#pragma unroll
        for (int k = 0; k < UPL; ++k) {
            if constexpr (EPU == 2) {
                // bfloat16 pairs: v_dot2_f32_bf16 (exact products, binary32 accumulation)
                x = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a[k]),
                                                    __builtin_bit_cast(bf16x2_t, b[j][k]), x, false);
            } else {
                x = fmaf(val<TT>(a[k], 0), val<TT>(b[j][k], 0), x);
            }
        }
        gj[j] = x;
    }
#pragma unroll
    for (int j = 0; j <= KMAX; ++j) gj[j] = group_sum<LPS>(gj[j]);
    if constexpr (LPS > KMAX) {
        // Every lane of the group holds all 1 + K dot products: lane gl takes slot gl's
        // sigmoid (one exp and one reciprocal per lane instead of 1 + K), and the step
        // sizes are then read back from lanes 0..K of the group.
        float xs = gj[0];
#pragma unroll
        for (int j = 1; j <= KMAX; ++j) xs = gl == j ? gj[j] : xs;
        const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-xs));
        const float gg = gl == 0 ? eta * (1.0f - sg) : -eta * g.alpha * sg;
#pragma unroll
        for (int j = 0; j <= KMAX; ++j) gj[j] = (FULL || j <= K) ? group_lane<LPS>(gg, j) : 0.f;
    } else {
#pragma unroll
        for (int j = 0; j <= KMAX; ++j) {
            float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-gj[j]));
            float gg = j == 0 ? eta * (1.0f - sg) : -eta * g.alpha * sg;
            gj[j] = j <= K ? gg : 0.f;
        }
    }
    const float el = eta * g.lambda;

    // dA = sum_j g_j b_j - (1 + K) eta lambda a
    float dA[UPL][EPU];
    const float decayA = (float)(K + 1) * el;
#pragma unroll
    for (int k = 0; k < UPL; ++k)
#pragma unroll
        for (int e = 0; e < EPU; ++e) {
            float acc = -decayA * val<TT>(a[k], e);
#pragma unroll
            for (int j = 0; j <= KMAX; ++j) acc = fmaf(gj[j], val<TT>(b[j][k], e), acc);
            dA[k][e] = acc;
        }

    if constexpr (SNAP) {
        // Entries of this sample/order: slot 0 = A[u] (dA), slot 1 + j = B[ids[j]] (delta_j).
        const unsigned long long e0 =
            ((s - so.base) * (unsigned long long)so.nord + (unsigned long long)oi) * (unsigned long long)(K + 2);
        float *crow = so.contrib + e0 * (unsigned long long)d;
#pragma unroll
        for (int k = 0; k < UPL; ++k) {
            const int un = k * LPS + gl;
            if (un < nu) {
#pragma unroll
                for (int e = 0; e < EPU; ++e) crow[un * EPU + e] = dA[k][e];
            }
        }
#pragma unroll
        for (int j = 0; j <= KMAX; ++j) {
            if (j > K) break;
            float *brow = crow + (unsigned long long)(j + 1) * d;
#pragma unroll
            for (int k = 0; k < UPL; ++k) {
                const int un = k * LPS + gl;
                if (un < nu) {
#pragma unroll
                    for (int e = 0; e < EPU; ++e) brow[un * EPU + e] = gj[j] * val<TT>(a[k], e) - el * val<TT>(b[j][k], e);
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
        // A row that occurs more than once in this order of the sample (two slots with
        // one row, or in first order a slot equal to the vertex row) takes the atomic
        // path at every occurrence: each occurrence adds its own increment, computed from
        // the rows as they were before the sample, so the row receives their sum.
        unsigned atom = hot | (dupb << 1);
        if constexpr (FIRST) atom |= (dupu << 1) | (dupu ? 1u : 0u);
        // bfloat16: the sample's seed for this order; slot q's row uses seed + (q + 1) c
        uint32_t seed = 0u;
        if constexpr (EPU == 2) seed = lowbias32(sr);
        constexpr uint32_t kSlot = 0x632BE59Bu;
        (void)oi;
        // vertex row
        write_row<TT, LPS, UPL, SH, FULL>(g, tabA, u, gl, a, dA, (atom & 1u) != 0, seed + kSlot);
        // context rows
#pragma unroll
        for (int j = 0; j <= KMAX; ++j) {
            if (!FULL && j > K) break;
            float inc[UPL][EPU];
#pragma unroll
            for (int k = 0; k < UPL; ++k)
#pragma unroll
                for (int e = 0; e < EPU; ++e) inc[k][e] = gj[j] * val<TT>(a[k], e) - el * val<TT>(b[j][k], e);
            write_row<TT, LPS, UPL, SH, FULL>(g, tabB, ids[j], gl, b[j], inc, (atom & (2u << j)) != 0,
                                        seed + (uint32_t)(j + 2) * kSlot);
        }
    }
}

// One tile of 64 samples [tile, min(tile + 64, end)).  UPL units per lane.  SH: bfloat16
// Hogwild with a binary32 shadow of the hot rows (compiled out otherwise: the shadow's
// address choice and second-half loads cost a quarter of the kernel's speed even unused).
template <typename TT, int LPS, int UPL, int KMAX, int ORD, bool SNAP, bool SH, bool FULL = false>
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
    unsigned my_dup = 0, my_hot = 0;
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
            const SlotDraw de = draw_slot(g, s, 0, slot0_columns(g));
            uint4 r0, r1;
            load_pair_rec<sizeof(TT) == 2>(g, s, de.col, de.x1, r0, r1);
            my_sr = (uint32_t)de.x2;
            __builtin_amdgcn_sched_barrier(0);
            SlotDraw dn[KMAX];
            uint4 nr[KMAX];
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < K) {
                    dn[j] = draw_slot(g, s, j + 1, g.n);
                    nr[j] = *reinterpret_cast<const uint4 *>(g.nrec + dn[j].col);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            my_eta = (float)(g.eta0 * (1.0 - (double)s / (double)g.T)) * g.eta_scale;
            const unsigned hh = (unsigned)g.hot_heat;  // -1 wraps to "nothing is that cold"
            const bool keep = edge_pick(r0, r1, de.x1, my_u, my_ids[0]);
            const unsigned eh = r1.w;  // heats: src_c, dst_c, src_a, dst_a
            const unsigned hu = keep ? (eh & 0xffu) : ((eh >> 16) & 0xffu);
            const unsigned hv = keep ? ((eh >> 8) & 0xffu) : (eh >> 24);
            if (g.hot_heat >= 0) my_hot = (hu <= hh ? 1u : 0u) | (hv <= hh ? 2u : 0u);
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < K) {
                    const bool kc = neg_pick(nr[j], dn[j], my_ids[j + 1]);
                    const unsigned hn = kc ? (nr[j].w & 0xffu) : ((nr[j].w >> 8) & 0xffu);
                    if (g.hot_heat >= 0 && hn <= hh) my_hot |= 4u << j;
                }
            }
            // low half: slots whose row occurs in another slot too (every occurrence);
            // high half: slots whose row is the vertex row u
#pragma unroll
            for (int j = 0; j <= KMAX; ++j) {
                if (j > K) break;
                if (my_ids[j] == my_u) my_dup |= 1u << (16 + j);
#pragma unroll
                for (int jj = 0; jj < j; ++jj)
                    if (my_ids[jj] == my_ids[j]) my_dup |= (1u << j) | (1u << jj);
            }
            // bfloat16 Hogwild with a shadow: the rows with a shadow slot are this launch's
            // hot rows; their ids become ~slot (negative, so equal rows stay equal and never
            // meet a table id).
            if constexpr (sizeof(TT) == 2 && !SNAP && SH) {
                if (g.slot) {
                    my_hot = 0;
                    int sl[KMAX + 2];
                    sl[0] = g.slot[my_u];
#pragma unroll
                    for (int j = 0; j <= KMAX; ++j) sl[j + 1] = j <= K ? g.slot[my_ids[j]] : -1;
                    if (sl[0] >= 0) {
                        my_u = ~sl[0];
                        my_hot |= 1u;
                    }
#pragma unroll
                    for (int j = 0; j <= KMAX; ++j)
                        if (sl[j + 1] >= 0) {
                            my_ids[j] = ~sl[j + 1];
                            my_hot |= 2u << j;
                        }
                }
            }
        }
    }

    // ---- phase B: LPS lanes per sample ----------------------------------------
    for (int r = 0; r < LPS; ++r) {
        const int src = r * GPW + grp;
        const int u = sample_lane<LPS>(my_u, src);
        int ids[KMAX + 1];
#pragma unroll
        for (int j = 0; j <= KMAX; ++j) ids[j] = sample_lane<LPS>(my_ids[j], src);
        const unsigned dup = (unsigned)sample_lane<LPS>((int)my_dup, src);
        unsigned hot = 0;
        uint32_t sr = 0;
        if constexpr (!SNAP) hot = (unsigned)sample_lane<LPS>((int)my_hot, src);
        if constexpr (sizeof(TT) == 2 && !SNAP) sr = (uint32_t)sample_lane<LPS>((int)my_sr, src);
        // every cross-lane read before lanes diverge
        const float eta = __int_as_float(sample_lane<LPS>(__float_as_int(my_eta), src));
        const unsigned long long s = tile + (unsigned long long)src;
        if (s >= end) continue;
        const unsigned dupb = dup & 0xffffu, dupu = dup >> 16;
        // Issue the row loads of both orders before any arithmetic or store, so that up to
        // 2 (2 + K) rows per sample are in flight at once.
        Rows<TT, UPL, KMAX> r2, r1;
        if constexpr ((ORD & 2) != 0)
            load_rows<TT, LPS, UPL, KMAX, SH, FULL>(r2, g, LH_TABLE_U, LH_TABLE_C, u, ids, K, gl);
        if constexpr ((ORD & 1) != 0)
            load_rows<TT, LPS, UPL, KMAX, SH, FULL>(r1, g, LH_TABLE_U1, LH_TABLE_U1, u, ids, K, gl);
        int oi = 0;
        if constexpr ((ORD & 2) != 0) {
            sgd_order<TT, LPS, UPL, KMAX, false, SNAP, SH, FULL>(g, u, ids, K, eta, dupb, dupu, hot, sr, oi, gl, so, s,
                                                       LH_TABLE_U, LH_TABLE_C, r2);
            ++oi;
        }
        if constexpr ((ORD & 1) != 0) {
            sgd_order<TT, LPS, UPL, KMAX, true, SNAP, SH, FULL>(g, u, ids, K, eta, dupb, dupu, hot, sr ^ 0x5bd1e995u, oi, gl,
                                                      so, s, LH_TABLE_U1, LH_TABLE_U1, r1);
        }
    }
}

}  // namespace lh
