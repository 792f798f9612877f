// Hogwild and SNAPSHOT-contribution kernels over a range of sample indices, and their
// host launchers.  Each (dtype, orders) pair is instantiated in its own translation
// unit so the kernel variants compile in parallel.
#pragma once

#include <algorithm>
#include <cmath>

#include "tile.hpp"

namespace lh {

// Register budget of the one-graph kernel: at least 3 (binary32) or 5 (bfloat16) waves per
// SIMD.  The bfloat16 kernel is latency bound: 5 waves (96 registers, no spills) measured
// 2 % faster than 4 on both hub-heavy and large uniform tables, and 6 (with spills) slower.
template <typename TT>
constexpr int hogwild_min_waves() { return sizeof(TT) == 2 ? 5 : 3; }

// SH: bfloat16 tables whose hot rows live in a binary32 shadow for the launch.  Each
// wavefront takes 64-sample tiles from the launch's tile counter (g.tiles, zero at launch)
// until none are left, so wavefronts that meet slow rows do not hold up a fixed share of
// the work and the grid is only as large as what is resident.
// FULL: the tile shape covers a row exactly (lanes x units == the row's units) and K == KMAX,
// so row accesses need no bounds mask or slot test.
template <typename TT, int LPS, int UPL, int KMAX, int ORD, bool SH, bool FULL = false>
__global__ void __launch_bounds__(256, hogwild_min_waves<TT>()) k_hogwild(GraphDev g, unsigned long long first, unsigned long long end)
{
    const unsigned lane = threadIdx.x & 63u;
    const unsigned long long ntiles = (end - first + 63) / 64;
    SnapOut so{};
    while (true) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(g.tiles, 1ull);
        t = ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(t >> 32)) << 32) |
            (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(t & 0xffffffffull));
        if (t >= ntiles) break;
        sgd_tile<TT, LPS, UPL, KMAX, ORD, false, SH, FULL>(g, first + t * 64, end, so);
    }
}

// Zero a launch's tile counter (a kernel, not a memset, so the launch can be captured).
template <int N>
__global__ void k_zero_tiles(unsigned long long *c)
{
    if (threadIdx.x < N) c[threadIdx.x] = 0ull;
}

template <typename TT, int LPS, int UPL, int KMAX, int ORD>
__global__ void __launch_bounds__(256) k_snap_contrib(GraphDev g, unsigned long long first, unsigned long long end,
                                                      SnapOut so)
{
    const unsigned wpb = blockDim.x >> 6;
    unsigned long long wave = (unsigned long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    unsigned long long nw = (unsigned long long)gridDim.x * wpb;
    unsigned long long ntiles = (end - first + 63) / 64;
    for (unsigned long long t = wave; t < ntiles; t += nw)
        sgd_tile<TT, LPS, UPL, KMAX, ORD, true, false>(g, first + t * 64, end, so);
}

inline unsigned hogwild_grid(unsigned long long count, int num_cu, int blocks_per_cu)
{
    unsigned long long tiles = (count + 63) / 64;
    unsigned long long blocks = (tiles + 3) / 4;
    unsigned long long cap = (unsigned long long)num_cu * (unsigned long long)(blocks_per_cu > 0 ? blocks_per_cu : 8);
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return (unsigned)blocks;
}

// Resident workgroups of a kernel on the device (at least 1 per CU).
template <typename KernelT>
inline unsigned resident_blocks(KernelT kernel, int num_cu)
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 256, 0) != hipSuccess || occ < 1) occ = 1;
    return (unsigned)num_cu * (unsigned)occ;
}

// Heat threshold for a launch whose rows are exposed to a window of W samples (those in
// flight, or unbounded for tables that fit in one L2): a row is hot when W p_r reaches
// hot_rate, i.e. when floor(-log2 p_r) <= floor(log2(W / hot_rate)).  hot_rate <= 0 makes
// every row hot, hot_rate >= 1e30 none.
inline int hot_heat_for(double W, double hot_rate)
{
    if (!(hot_rate > 0.0)) return 255;
    if (hot_rate >= 1e30 || !(W > 0.0)) return -1;
    if (std::isinf(W)) return 255;
    double t = std::floor(std::log2(W / hot_rate));
    if (t < -1.0) return -1;
    if (t > 255.0) return 255;
    return (int)t;
}

// Samples in flight in phase B: resident wavefronts x (64 / LPS) groups.
template <typename KernelT>
inline double samples_in_flight(KernelT kernel, unsigned grid, int num_cu, int lps)
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 256, 0) != hipSuccess || occ < 1) occ = 8;
    double blocks = std::min<double>((double)grid, (double)num_cu * occ);
    return blocks * 4.0 * (64.0 / lps);
}

// (lanes per sample, units per lane) of the Hogwild kernels.
#define LH_CFG_LIST(X) \
    X(16, 1)           \
    X(32, 1)           \
    X(64, 1)           \
    X(16, 2)           \
    X(32, 2)           \
    X(64, 2)           \
    X(2, 4)            \
    X(4, 4)            \
    X(8, 4)            \
    X(16, 4)           \
    X(32, 4)           \
    X(64, 4)           \
    X(4, 8)            \
    X(8, 8)            \
    X(16, 8)           \
    X(32, 8)           \
    X(64, 8)

// SNAPSHOT contributions use only the natural configuration of each width.
#define LH_SNAP_CFG_LIST(X) \
    X(2, 4)                 \
    X(4, 4)                 \
    X(8, 4)                 \
    X(16, 4)                \
    X(32, 4)                \
    X(64, 4)                \
    X(64, 8)

// The grid of one Hogwild launch over `count` samples and the samples it keeps in flight:
// the configuration's grid, lowered if the graph's staleness cap asks for fewer.
template <typename KernelT>
inline double plan_launch(KernelT kern, int lps, const GraphDev &g, const TileCfg &c, unsigned long long count,
                          int num_cu, unsigned *grid_out)
{
    unsigned grid = std::min(hogwild_grid(count, num_cu, c.blocks_per_cu), resident_blocks(kern, num_cu));
    double F = samples_in_flight(kern, grid, num_cu, lps);
    if (g.max_in_flight > 0.0 && F > g.max_in_flight) {
        double per_block = 4.0 * (64.0 / lps);
        grid = (unsigned)std::max(1.0, std::floor(g.max_in_flight / per_block));
        F = samples_in_flight(kern, grid, num_cu, lps);
    }
    *grid_out = grid;
    return F;
}

// One Hogwild launch with the heat threshold for its concurrency.  With a shadow context
// (bfloat16 tables) the hot rows move into the binary32 shadow for the launch and back
// afterwards; without one no row is read from a shadow.
template <typename KernelT>
hipError_t launch_one(KernelT kern, int lps, const GraphDev &g, const TileCfg &c, unsigned long long first,
                      unsigned long long end, int num_cu, const ShadowCtx *sc, hipStream_t s)
{
    unsigned grid = 0;
    const double F = plan_launch(kern, lps, g, c, end - first, num_cu, &grid);
    GraphDev gl = g;
    gl.hot_heat = hot_heat_for(F + g.resid, g.hot_rate);
    if (sc) {
        hipError_t e = shadow_begin(*sc, gl.hot_heat, s);
        if (e != hipSuccess) return e;
    } else {
        gl.slot = nullptr;
    }
    if (!gl.tiles) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_tiles<1>, dim3(1), dim3(64), 0, s, gl.tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, gl, first, end);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && sc) e = shadow_end(*sc, gl.hot_heat, first, s);
    return e;
}

// Samples a Hogwild launch of `count` samples would keep in flight (0: no such kernel);
// g.slot set means the kernel with the binary32 shadow (bfloat16 only).
template <typename TT, int ORD, bool SH>
double hogwild_in_flight_sh(const GraphDev &g, const TileCfg &c, unsigned long long count, int num_cu)
{
    unsigned grid = 0;
#define LH_PLAN_H(L, C)                                                                                  \
    if (c.lps == L && c.upl == C) {                                                                      \
        if (!SH && g.K == 5 && L * C == g.nunits)                                                        \
            return plan_launch(k_hogwild<TT, L, C, 5, ORD, false, true>, L, g, c, count, num_cu, &grid);   \
        return plan_launch(g.K <= 5 ? k_hogwild<TT, L, C, 5, ORD, SH> : k_hogwild<TT, L, C, 8, ORD, SH>, L, g, c, \
                           count, num_cu, &grid);                                                        \
    }
    LH_CFG_LIST(LH_PLAN_H)
#undef LH_PLAN_H
    return 0.0;
}

template <typename TT, int ORD>
double hogwild_in_flight_t(const GraphDev &g, const TileCfg &c, unsigned long long count, int num_cu)
{
    if constexpr (sizeof(TT) == 2)
        if (g.slot) return hogwild_in_flight_sh<TT, ORD, true>(g, c, count, num_cu);
    return hogwild_in_flight_sh<TT, ORD, false>(g, c, count, num_cu);
}

template <typename TT, int ORD, bool SH>
hipError_t launch_hogwild_sh(const GraphDev &g, const TileCfg &c, unsigned long long first, unsigned long long end,
                             int num_cu, const ShadowCtx *sc, hipStream_t s)
{
    const bool k5 = g.K <= 5;
#define LH_LAUNCH_H(L, C)                                                                        \
    if (c.lps == L && c.upl == C) {                                                              \
        if (!SH && g.K == 5 && L * C == g.nunits)                                                \
            return launch_one(k_hogwild<TT, L, C, 5, ORD, false, true>, L, g, c, first, end, num_cu, sc, s); \
        if (k5) return launch_one(k_hogwild<TT, L, C, 5, ORD, SH>, L, g, c, first, end, num_cu, sc, s); \
        return launch_one(k_hogwild<TT, L, C, 8, ORD, SH>, L, g, c, first, end, num_cu, sc, s);        \
    }
    LH_CFG_LIST(LH_LAUNCH_H)
#undef LH_LAUNCH_H
    return hipErrorInvalidConfiguration;
}

// A shadow context selects the kernel built with the shadow path (bfloat16 only).
template <typename TT, int ORD>
hipError_t launch_hogwild_t(const GraphDev &g, const TileCfg &c, unsigned long long first, unsigned long long end,
                            int num_cu, const ShadowCtx *sc, hipStream_t s)
{
    if constexpr (sizeof(TT) == 2)
        if (sc) return launch_hogwild_sh<TT, ORD, true>(g, c, first, end, num_cu, sc, s);
    return launch_hogwild_sh<TT, ORD, false>(g, c, first, end, num_cu, nullptr, s);
}

template <typename TT, int ORD>
hipError_t launch_snap_t(const GraphDev &g, const TileCfg &c, unsigned long long first, unsigned long long end,
                         int num_cu, const SnapOut &so, hipStream_t s)
{
    const bool k5 = g.K <= 5;
    dim3 grid(hogwild_grid(end - first, num_cu, 8)), block(256);
#define LH_LAUNCH_S(L, C)                                                                              \
    if (c.lps == L && c.upl == C) {                                                                    \
        if (k5)                                                                                        \
            hipLaunchKernelGGL((k_snap_contrib<TT, L, C, 5, ORD>), grid, block, 0, s, g, first, end, so); \
        else                                                                                           \
            hipLaunchKernelGGL((k_snap_contrib<TT, L, C, 8, ORD>), grid, block, 0, s, g, first, end, so); \
        return hipGetLastError();                                                                      \
    }
    LH_SNAP_CFG_LIST(LH_LAUNCH_S)
#undef LH_LAUNCH_S
    return hipErrorInvalidConfiguration;
}

// Explicit instantiations live in sgd_<dtype>_o<orders>.hip.
#define LH_DECLARE_LAUNCHERS(TT, ORD)                                                                          \
    extern template hipError_t launch_hogwild_t<TT, ORD>(const GraphDev &, const TileCfg &, unsigned long long, \
                                                         unsigned long long, int, const ShadowCtx *, hipStream_t); \
    extern template hipError_t launch_snap_t<TT, ORD>(const GraphDev &, const TileCfg &, unsigned long long,    \
                                                      unsigned long long, int, const SnapOut &, hipStream_t); \
    extern template double hogwild_in_flight_t<TT, ORD>(const GraphDev &, const TileCfg &, unsigned long long, int);

#define LH_DEFINE_LAUNCHERS(TT, ORD)                                                                    \
    template hipError_t launch_hogwild_t<TT, ORD>(const GraphDev &, const TileCfg &, unsigned long long, \
                                                  unsigned long long, int, const ShadowCtx *, hipStream_t); \
    template hipError_t launch_snap_t<TT, ORD>(const GraphDev &, const TileCfg &, unsigned long long,    \
                                               unsigned long long, int, const SnapOut &, hipStream_t); \
    template double hogwild_in_flight_t<TT, ORD>(const GraphDev &, const TileCfg &, unsigned long long, int);

}  // namespace lh
