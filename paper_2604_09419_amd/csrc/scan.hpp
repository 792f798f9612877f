// Canonical chunked inclusive scan on the GPU.
//
// The association order is fixed: chunk c covers [c*1024, min((c+1)*1024, n)); one
// thread runs the chunk's left-to-right chain; the chunk totals are scanned the same
// way, recursively; element i of chunk c > 0 becomes combine(inc[c-1], loc[i]).  For
// the binary64 compensated sum this order is part of the definition of the alias
// tables' normalisation and prefix sums, so the GPU result is bitwise reproducible
// against any implementation of the same definition.  For max and for integer sums
// the order does not matter, and the same code is reused.
//
// This header is compiled only into translation units built with -ffp-contract=off.
#pragma once

#include "common.hpp"

namespace lh {

constexpr int SCAN_CHUNK = 1024;

// Neumaier-compensated running sum; the chunk value is s + comp after each element.
struct OpNeumaier {
    using T = double;
    struct State {
        double s, c;
    };
    __device__ static State init() { return State{0.0, 0.0}; }
    __device__ static double step(State &st, double x)
    {
        double t = st.s + x;
        if (fabs(st.s) >= fabs(x))
            st.c += (st.s - t) + x;
        else
            st.c += (x - t) + st.s;
        st.s = t;
        return st.s + st.c;
    }
    __device__ static double combine(double off, double loc) { return off + loc; }
};

struct OpMax {
    using T = double;
    struct State {
        double m;
    };
    __device__ static State init() { return State{-__builtin_huge_val()}; }
    __device__ static double step(State &st, double x)
    {
        st.m = x > st.m ? x : st.m;
        return st.m;
    }
    __device__ static double combine(double off, double loc) { return loc > off ? loc : off; }
};

template <class I>
struct OpAdd {
    using T = I;
    struct State {
        I s;
    };
    __device__ static State init() { return State{I(0)}; }
    __device__ static I step(State &st, I x)
    {
        st.s += x;
        return st.s;
    }
    __device__ static I combine(I off, I loc) { return off + loc; }
};

// Elements a chain loads ahead of its arithmetic: the chain itself is one dependent
// sequence, but its loads are not, so they are issued in blocks of this many.
constexpr int CHAIN_BLOCK = 64;

// The left-to-right chain of one chunk [lo, hi), in place or not (each block is loaded
// before any of its results is stored).
template <class Op>
__device__ __forceinline__ typename Op::T chain(const typename Op::T *x, typename Op::T *out, long long lo,
                                                long long hi)
{
    typename Op::State st = Op::init();
    typename Op::T last{};
    long long i = lo;
    for (; i + CHAIN_BLOCK <= hi; i += CHAIN_BLOCK) {
        typename Op::T v[CHAIN_BLOCK];
#pragma unroll
        for (int k = 0; k < CHAIN_BLOCK; ++k) v[k] = x[i + k];
#pragma unroll
        for (int k = 0; k < CHAIN_BLOCK; ++k) {
            last = Op::step(st, v[k]);
            out[i + k] = last;
        }
    }
    for (; i < hi; ++i) {
        last = Op::step(st, x[i]);
        out[i] = last;
    }
    return last;
}

template <class Op>
__global__ void __launch_bounds__(256) k_chunk_chain(const typename Op::T *x, typename Op::T *out,
                                                     long long n, typename Op::T *tot)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long nch = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (c >= nch) return;
    long long lo = c * SCAN_CHUNK, hi = lo + SCAN_CHUNK < n ? lo + SCAN_CHUNK : n;
    tot[c] = chain<Op>(x, out, lo, hi);
}

template <class Op>
__global__ void __launch_bounds__(256) k_chunk_offset(typename Op::T *out, long long n,
                                                      const typename Op::T *inc)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long long c = i / SCAN_CHUNK;
    if (c == 0) return;
    out[i] = Op::combine(inc[c - 1], out[i]);
}

// Elements of level storage needed for a scan of n items.
static inline long long scan_levels_size(long long n)
{
    long long total = 0;
    while (n > 1) {
        n = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
        total += n;
    }
    return total + 8;
}

// Inclusive scan of x[0..n) into out (out may equal x).  levels must hold
// scan_levels_size(n) elements.
template <class Op>
static void chunk_scan(const typename Op::T *x, typename Op::T *out, long long n,
                       typename Op::T *levels, hipStream_t s)
{
    if (n <= 0) return;
    long long nch = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    hipLaunchKernelGGL(k_chunk_chain<Op>, dim3((unsigned)LH_CDIV(nch, 256)), dim3(256), 0, s, x, out,
                       n, levels);
    if (nch > 1) {
        chunk_scan<Op>(levels, levels, nch, levels + nch, s);
        hipLaunchKernelGGL(k_chunk_offset<Op>, dim3((unsigned)LH_CDIV(n, 256)), dim3(256), 0, s, out,
                           n, levels);
    }
}

}  // namespace lh
