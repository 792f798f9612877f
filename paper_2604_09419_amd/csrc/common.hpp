// Shared device and host helpers of the linehip library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "linehip.h"

// ---------------------------------------------------------------------------
// Record layouts in HBM.
//
// Edge alias record (32 B, one per arc column c): the 64-bit threshold, the alias
// arc, the endpoints of both the column arc and the alias arc (so that one 32-byte
// sector read resolves a positive pair with no dependent load), and the heat byte of
// each of those four endpoints.
// Negative alias record (16 B, one per node column): threshold, alias, and the heat
// bytes of the column node (byte 0) and of the alias node (byte 1).
//
// Heat of node r: floor(-log2 p_r), clamped to [0, 255], where p_r estimates the
// probability that one sample touches a row of r: (out-degree + in-degree) / m plus
// K q(r) with q from Eq. (1).  A training launch with F samples in flight treats a row
// as hot when F p_r reaches the caller's threshold, i.e. when its heat is at most
// floor(log2(F / threshold)).
// ---------------------------------------------------------------------------
struct __attribute__((aligned(16))) EdgeRec {
    unsigned long long thr;
    int32_t alias;
    int32_t src_c;
    int32_t dst_c;
    int32_t src_a;
    int32_t dst_a;
    uint32_t heat;
};
static_assert(sizeof(EdgeRec) == 32, "EdgeRec is one 32-byte sector");

struct __attribute__((aligned(16))) NegRec {
    unsigned long long thr;
    int32_t alias;
    uint32_t heat;
};
static_assert(sizeof(NegRec) == 16, "NegRec is 16 bytes");

// One entry of a walk row (the neighbourhood N(x) of the walk graph): the alias table
// of discrete(N(x)) with both outcomes resolved to vertices, so one 16-byte read decides
// a step: the entry keeps its own head when the draw's threshold word is below thr, else
// it yields the head of its alias entry.
struct __attribute__((aligned(16))) WalkRec {
    unsigned long long thr;
    int32_t keep;   // head of this entry
    int32_t alias;  // head of the alias entry
};
static_assert(sizeof(WalkRec) == 16, "WalkRec is 16 bytes");

// Device status word bits (accumulated with atomicOr, read by lh_check).
enum : unsigned int {
    ST_OUT_OF_RANGE = 1u,
    ST_BAD_WEIGHT = 2u,
    ST_ZERO_TOTAL = 4u,
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the 4x64 S-box,
// key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct u64x4 {
    unsigned long long x, y, z, w;
};

__device__ __forceinline__ u64x4 philox4x64_10(unsigned long long k0, unsigned long long k1,
                                               unsigned long long c0, unsigned long long c1,
                                               unsigned long long c2, unsigned long long c3)
{
    const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        unsigned long long hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        unsigned long long hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        unsigned long long n0 = hi1 ^ c1 ^ k0;
        unsigned long long n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return u64x4{c0, c1, c2, c3};
}

// Column of a draw: floor(x0 * N / 2^64).
__device__ __forceinline__ long long draw_column(unsigned long long x0, long long N)
{
    return (long long)__umul64hi(x0, (unsigned long long)N);
}

// lowbias32 integer hash (C. Wellons, "Prospecting for hash functions", 2018): used to
// expand one Philox word into the per-element bits of stochastic rounding.
__device__ __forceinline__ uint32_t lowbias32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// ---------------------------------------------------------------------------
// bfloat16 helpers.  Loads widen exactly; init uses round-to-nearest-even; training
// write-back uses stochastic rounding: add 16 random bits to the binary32 pattern and
// keep the high half (NaN passes through as a quiet NaN).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h16)
{
    return __uint_as_float(h16 << 16);
}

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
    uint32_t lsb = (u >> 16) & 1u;
    return (u + 0x7fffu + lsb) >> 16;
}

// Two binary32 values as one packed bfloat16 pair, element 0 in the low half.
// Stochastic rounding: element 0 adds bits 0-15 of rnd to its binary32 pattern and keeps
// the high half, element 1 adds bits 16-31 (NaN stays NaN).  gfx950's v_cvt_sr_bf16_f32
// adds the high 16 bits of its random operand (measured on MI355X for every finite input,
// denormals included), one instruction per element.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t bf16x2_sr(float x0, float x1, uint32_t rnd)
{
    bf16x2_t v = {};
    v = __builtin_amdgcn_cvt_sr_bf16_f32(v, x0, rnd << 16, false);
    v = __builtin_amdgcn_cvt_sr_bf16_f32(v, x1, rnd, true);
    return __builtin_bit_cast(uint32_t, v);
}

// Round to nearest even: one v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t bf16x2_rne(float x0, float x1)
{
    const bf16x2_t v = {(__bf16)x0, (__bf16)x1};
    return __builtin_bit_cast(uint32_t, v);
}

// ---------------------------------------------------------------------------
// Host-side helpers.
// ---------------------------------------------------------------------------
#define LH_CDIV(a, b) (((a) + (b)-1) / (b))

static inline size_t lh_align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
