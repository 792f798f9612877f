// Canonical chunked scans of many segments of one array at once.
//
// Segment s covers [start[s], start[s] + len[s]) and is scanned exactly as the canonical
// scan of scan.hpp scans an array of its own: chunks of SCAN_CHUNK counted from the
// segment's start, one left-to-right chain per chunk, the chunk totals of the segment
// scanned the same way (recursively), and element i of chunk j > 0 becoming
// combine(inc[j - 1], loc[i]).  So every segment's binary64 compensated sums are bitwise
// the ones a scan of that segment alone gives.
//
// One level: the chunks of all segments are listed (chunk c of segment s at
// cb[s] + j, so a segment's chunks are consecutive), every chunk's chain runs in its own
// thread, and the totals of the segments with more than one chunk are scanned as the
// segments of the next level; then every chunk j > 0 adds its predecessor's scanned total.
//
// Compiled only into translation units built with -ffp-contract=off.
#pragma once

#include "scan.hpp"

namespace lh {

// Bump allocator over a caller's device scratch (256-byte granules).
struct Arena {
    char *base = nullptr;
    size_t bytes = 0, used = 0;
    template <class T>
    T *take(long long count)
    {
        size_t need = ((size_t)(count > 0 ? count : 1) * sizeof(T) + 255) & ~(size_t)255;
        if (used + need > bytes) return nullptr;
        T *p = reinterpret_cast<T *>(base + used);
        used += need;
        return p;
    }
};

__global__ void k_seg_nch(const long long *len, long long S, long long *nch)
{
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) nch[s] = (len[s] + SCAN_CHUNK - 1) / SCAN_CHUNK;
}

__global__ void k_seg_zero(unsigned long long *cnt, int k)
{
    if ((int)threadIdx.x < k) cnt[threadIdx.x] = 0ull;
}

// Chunk list of every segment; the chunks j > 0 are appended to `later` and the segments
// of more than one chunk (their totals' range in the next level) to lstart / llen.  The
// order of appends does not matter: each listed item is handled on its own.
__global__ void k_seg_chunks(const long long *start, const long long *len, const long long *nch,
                             const long long *cbi, long long S, long long *cstart, long long *cend,
                             long long *later, unsigned long long *nlater, long long *lstart, long long *llen,
                             unsigned long long *nlong)
{
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const long long k = nch[s], cb = cbi[s] - k, st = start[s], en = start[s] + len[s];
    for (long long j = 0; j < k; ++j) {
        const long long lo = st + j * SCAN_CHUNK;
        cstart[cb + j] = lo;
        cend[cb + j] = lo + SCAN_CHUNK < en ? lo + SCAN_CHUNK : en;
        if (j > 0) later[atomicAdd(nlater, 1ull)] = cb + j;
    }
    if (k > 1) {
        const unsigned long long i = atomicAdd(nlong, 1ull);
        lstart[i] = cb;
        llen[i] = k;
    }
}

template <class Op>
__global__ void __launch_bounds__(256) k_seg_chain(typename Op::T *x, const long long *cstart, const long long *cend,
                                                   long long NC, typename Op::T *tot)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= NC) return;
    tot[c] = chain<Op>(x, x, cstart[c], cend[c]);
}

// Listed chunks c (j > 0): element i becomes combine(inc[c - 1], loc[i]), with inc the
// scanned chunk totals.  A workgroup per listed chunk, grid-strided over the list.
template <class Op>
__global__ void __launch_bounds__(256) k_seg_offset(typename Op::T *x, const long long *cstart, const long long *cend,
                                                    const long long *later, const unsigned long long *nlater,
                                                    const typename Op::T *inc)
{
    const unsigned long long n = *nlater;
    for (unsigned long long b = blockIdx.x; b < n; b += gridDim.x) {
        const long long c = later[b];
        const typename Op::T off = inc[c - 1];
        for (long long i = cstart[c] + threadIdx.x; i < cend[c]; i += blockDim.x) x[i] = Op::combine(off, x[i]);
    }
}

// Device bytes seg_scan may take from its arena for S segments over E elements.
static inline size_t seg_scan_bytes(long long S, long long E)
{
    size_t total = 0;
    for (int level = 0; level < 8 && S > 0; ++level) {
        const long long NC = S + E / SCAN_CHUNK + 1;
        const long long SL = E / (SCAN_CHUNK + 1) + 1;
        total += 3 * (((size_t)S * 8 + 255) & ~(size_t)255);                         // nch, cbi, levels (bound)
        total += ((size_t)scan_levels_size(S) * 8 + 255) & ~(size_t)255;
        total += 4 * (((size_t)NC * 8 + 255) & ~(size_t)255);                        // cstart, cend, tot, later
        total += 2 * (((size_t)SL * 8 + 255) & ~(size_t)255) + 256;                  // lstart, llen, counters
        S = SL;
        E = NC;
    }
    return total + 4096;
}

// In-place canonical scan of S segments of x (E elements in all).  Synchronises the
// stream once per level (to size the chunk list).  Returns hipErrorOutOfMemory when the
// arena is too small.
template <class Op>
static hipError_t seg_scan(typename Op::T *x, long long E, const long long *start, const long long *len, long long S,
                           Arena &ar, hipStream_t st, int depth = 0)
{
    using T = typename Op::T;
    if (S <= 0 || E <= 0) return hipSuccess;
    if (depth > 8) return hipErrorInvalidValue;
    const size_t mark = ar.used;
    long long *nch = ar.take<long long>(S), *cbi = ar.take<long long>(S);
    long long *lev = ar.take<long long>(scan_levels_size(S));
    unsigned long long *cnt = ar.take<unsigned long long>(4);
    if (!nch || !cbi || !lev || !cnt) return hipErrorOutOfMemory;
    const unsigned gs = (unsigned)LH_CDIV(S, 256);
    hipLaunchKernelGGL(k_seg_nch, dim3(gs), dim3(256), 0, st, len, S, nch);
    chunk_scan<OpAdd<long long>>(nch, cbi, S, lev, st);
    long long NC = 0;
    hipError_t e = hipMemcpyAsync(&NC, cbi + (S - 1), sizeof(NC), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (NC <= 0) {
        ar.used = mark;
        return hipSuccess;
    }
    const long long SL = E / (SCAN_CHUNK + 1) + 1;  // segments of more than one chunk
    long long *cstart = ar.take<long long>(NC), *cend = ar.take<long long>(NC), *later = ar.take<long long>(NC);
    T *tot = ar.take<T>(NC);
    long long *lstart = ar.take<long long>(SL), *llen = ar.take<long long>(SL);
    if (!cstart || !cend || !later || !tot || !lstart || !llen) return hipErrorOutOfMemory;
    hipLaunchKernelGGL(k_seg_zero, dim3(1), dim3(64), 0, st, cnt, 4);
    hipLaunchKernelGGL(k_seg_chunks, dim3(gs), dim3(256), 0, st, start, len, nch, cbi, S, cstart, cend, later,
                       cnt + 0, lstart, llen, cnt + 1);
    hipLaunchKernelGGL(k_seg_chain<Op>, dim3((unsigned)LH_CDIV(NC, 256)), dim3(256), 0, st, x, cstart, cend, NC, tot);
    unsigned long long nlong = 0;
    e = hipMemcpyAsync(&nlong, cnt + 1, sizeof(nlong), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (nlong > 0) {
        e = seg_scan<Op>(tot, NC, lstart, llen, (long long)nlong, ar, st, depth + 1);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_seg_offset<Op>, dim3(2048), dim3(256), 0, st, x, cstart, cend, later, cnt + 0,
                           (const T *)tot);
    }
    e = hipGetLastError();
    ar.used = mark;
    return e;
}

}  // namespace lh
