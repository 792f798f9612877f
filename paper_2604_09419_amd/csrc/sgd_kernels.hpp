// Hogwild and SNAPSHOT-contribution kernels over a range of sample indices, and their
// host launchers.  Each (dtype, orders) pair is instantiated in its own translation
// unit so the kernel variants compile in parallel.
#pragma once

#include "tile.hpp"

namespace lh {

// Grid-stride over 64-sample tiles: wave w takes tiles w, w + W, w + 2W, ...
template <typename TT, int LPS, int CPL, int KMAX, int ORD>
__global__ void __launch_bounds__(256) k_hogwild(GraphDev g, unsigned long long first, unsigned long long end)
{
    const unsigned wpb = blockDim.x >> 6;
    unsigned long long wave = (unsigned long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    unsigned long long nw = (unsigned long long)gridDim.x * wpb;
    unsigned long long ntiles = (end - first + 63) / 64;
    SnapOut so{};
    for (unsigned long long t = wave; t < ntiles; t += nw)
        sgd_tile<TT, LPS, CPL, KMAX, ORD, false>(g, first + t * 64, end, so);
}

template <typename TT, int LPS, int CPL, int KMAX, int ORD>
__global__ void __launch_bounds__(256) k_snap_contrib(GraphDev g, unsigned long long first, unsigned long long end,
                                                      SnapOut so)
{
    const unsigned wpb = blockDim.x >> 6;
    unsigned long long wave = (unsigned long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    unsigned long long nw = (unsigned long long)gridDim.x * wpb;
    unsigned long long ntiles = (end - first + 63) / 64;
    for (unsigned long long t = wave; t < ntiles; t += nw)
        sgd_tile<TT, LPS, CPL, KMAX, ORD, true>(g, first + t * 64, end, so);
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

#define LH_CFG_LIST(X) \
    X(2, 1)            \
    X(4, 1)            \
    X(8, 1)            \
    X(16, 1)           \
    X(32, 1)           \
    X(64, 1)           \
    X(4, 2)            \
    X(8, 2)            \
    X(16, 2)           \
    X(32, 2)           \
    X(64, 2)

// SNAPSHOT contributions use only the natural configuration of each width.
#define LH_SNAP_CFG_LIST(X) \
    X(2, 1)                 \
    X(4, 1)                 \
    X(8, 1)                 \
    X(16, 1)                \
    X(32, 1)                \
    X(64, 1)                \
    X(64, 2)

template <typename TT, int ORD>
hipError_t launch_hogwild_t(const GraphDev &g, const TileCfg &c, unsigned long long first, unsigned long long end,
                            int num_cu, hipStream_t s)
{
    const bool k5 = g.K <= 5;
    dim3 grid(hogwild_grid(end - first, num_cu, c.blocks_per_cu)), block(256);
#define LH_LAUNCH_H(L, C)                                                                    \
    if (c.lps == L && c.cpl == C) {                                                          \
        if (k5)                                                                              \
            hipLaunchKernelGGL((k_hogwild<TT, L, C, 5, ORD>), grid, block, 0, s, g, first, end); \
        else                                                                                 \
            hipLaunchKernelGGL((k_hogwild<TT, L, C, 8, ORD>), grid, block, 0, s, g, first, end); \
        return hipGetLastError();                                                            \
    }
    LH_CFG_LIST(LH_LAUNCH_H)
#undef LH_LAUNCH_H
    return hipErrorInvalidConfiguration;
}

template <typename TT, int ORD>
hipError_t launch_snap_t(const GraphDev &g, const TileCfg &c, unsigned long long first, unsigned long long end,
                         int num_cu, const SnapOut &so, hipStream_t s)
{
    const bool k5 = g.K <= 5;
    dim3 grid(hogwild_grid(end - first, num_cu, 8)), block(256);
#define LH_LAUNCH_S(L, C)                                                                              \
    if (c.lps == L && c.cpl == C) {                                                                    \
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
                                                         unsigned long long, int, hipStream_t);                \
    extern template hipError_t launch_snap_t<TT, ORD>(const GraphDev &, const TileCfg &, unsigned long long,    \
                                                      unsigned long long, int, const SnapOut &, hipStream_t);

#define LH_DEFINE_LAUNCHERS(TT, ORD)                                                                    \
    template hipError_t launch_hogwild_t<TT, ORD>(const GraphDev &, const TileCfg &, unsigned long long, \
                                                  unsigned long long, int, hipStream_t);                \
    template hipError_t launch_snap_t<TT, ORD>(const GraphDev &, const TileCfg &, unsigned long long,    \
                                               unsigned long long, int, const SnapOut &, hipStream_t);

}  // namespace lh
