// Internal host-side state of a linehip handle and the workspace layouts.
#pragma once

#include <functional>
#include <string>

#include "common.hpp"

namespace lh {

// One graph as the training kernels see it (passed by value to kernels).
struct GraphDev {
    void *tab[3];              // U, C, U1 (binary32 or bfloat16), NULL when unused
    const EdgeRec *erec;       // [m]
    const NegRec *nrec;        // [n]
    long long m, n;
    unsigned long long seed;   // Philox key word 0
    unsigned long long key1;   // Philox key word 1 for sampling (graph_id)
    unsigned long long sr_key; // Philox key word 1 for stochastic-rounding bits
    unsigned long long T;
    double eta0;
    float lambda, alpha;
    float eta_scale;           // 1 for training, 0 for timing-only dry runs
    int d;                     // width
    int nunits;                // 4-byte units per row (d binary32 values or d/2 bfloat16 pairs)
    int K;
    int hot_heat;              // rows with heat <= hot_heat take atomic increments (-1: none)
    double hot_rate;           // host side: the threshold hot_heat is derived from per launch
    double max_in_flight;      // host side: cap on samples in flight (0: none)
    double resid;              // host side: extra hot window (infinite for tables that fit in one L2)
    // bfloat16 Hogwild: binary32 shadow rows of the hot rows ([cap x d] per table) and the
    // per-node slot map (slot >= 0: the row lives in the shadow for this launch).  NULL
    // for binary32 tables and SNAPSHOT.
    float *shadow[3];
    const int32_t *slot;
    // Hogwild: the launch's tile counter (device word, reset to 0 before each launch);
    // wavefronts take 64-sample tiles from it until none are left.
    unsigned long long *tiles;
    // Positive pairs from random walks: pairs[s - pairs_first] is the (u, v) of sample s
    // (every sample of the launch lies in the buffer); NULL: slot 0 draws an arc.  heat:
    // per-node heat, for the write path of a walk pair's rows.
    const int2 *pairs;
    unsigned long long pairs_first;
    const uint8_t *heat;
    // With pairs set and pool_n = R > 0: a pair pool instead, pairs[0 .. R) the collected
    // pairs, and sample s takes (pairs[i].x, pairs[j].y) with i, j slot 0's two column
    // draws over R.
    unsigned long long pool_n;
};

// The random-walk pair source of a handle (lh_walk_build).
struct WalkState {
    bool ready = false;
    int L = 0, W = 0;                 // walk length (vertices), window
    long long Bw = 0, P = 0;          // walks per batch, pairs per walk
    long long chunk_walks = 0;        // walks whose pairs one buffer fill holds (a multiple of Bw)
    long long *off = nullptr;         // [n + 1] row offsets of the walk graph
    WalkRec *rec = nullptr;           // [2m] row entries
    int2 *pairs = nullptr;            // [chunk_walks * P]
    long long loaded = -1;            // the chunk the buffer holds (-1: none)
    unsigned long long pool = 0;      // pair pool: its R collected pairs (chunk 0's first R); 0: none
};

// Persistent walk memory: offsets, records, pair buffer (256-byte aligned pieces).
struct WalkLayout {
    size_t off = 0, rec = 0, pairs = 0, total = 0;
    long long chunk_walks = 0, P = 0;
};
WalkLayout walk_layout(long long n, long long m, int L, int W, long long Bw);

// A kernel configuration: lanes per sample, 4-byte units of a row per lane (a unit is one
// binary32 value or two bfloat16 values) and workgroups per compute unit.
struct TileCfg {
    int lps = 0, upl = 0, blocks_per_cu = 0;
};

struct WsLayout {
    size_t status = 0, tiles = 0, erec = 0, nrec = 0;
    size_t nheat = 0;                                   // [n] bytes: per-node heat
    size_t slot = 0, srows = 0, shadow = 0;             // bfloat16 Hogwild shadow (else 0)
    long long shadow_cap = 0;                           // shadow rows per table
    size_t keys0 = 0, keys1 = 0, vals0 = 0, vals1 = 0, contrib = 0, hist = 0, ilev = 0,
           seg = 0, segid = 0, total = 0;
    long long entries = 0, hist_n = 0, ilev_n = 0;
};

struct ScratchLayout {
    size_t wq = 0, dx = 0, idx = 0, lpos = 0, deg = 0, indeg = 0, cnt = 0, lev = 0, ilev = 0, total = 0;
    long long N = 0, lev_n = 0;
};

WsLayout ws_layout(const lh_params &p, long long n, long long m);

// bfloat16 Hogwild handles that ask for it (hot_shadow = 1) keep their hot rows in a
// binary32 shadow.  (Binary32 handles apply their atomics to the table rows: a compact
// shadow measured no faster for them.)
inline bool uses_shadow(const lh_params &p) { return p.mode == LH_HOGWILD && p.dtype == LH_BF16 && p.hot_shadow == 1; }

// Shadow rows per table of a Hogwild handle with a shadow and n nodes: every node of a graph
// of up to 2^17 nodes, else one node in 16.  The hot set of a launch is trimmed to fit.
inline long long shadow_capacity(long long n)
{
    long long c = (n + 15) / 16;
    if (c < (1ll << 17)) c = 1ll << 17;
    return c < n ? c : n;
}

// Host view of one handle's shadow for a launch (see shadow_begin / shadow_end).
struct ShadowCtx {
    const uint8_t *nheat;       // [n] per-node heat
    int32_t *slot;              // [n]
    int32_t *srows;             // [cap] node of each slot
    float *shadow[3];           // [cap x d] per table, NULL when the table is unused
    void *tab[3];               // the bfloat16 tables
    unsigned int *counter;      // device word: slots handed out
    const unsigned long long *heat_count;  // host [256]: nodes per heat value
    long long n, cap;
    int d;
    unsigned long long seed, sr_key;
};

// Extra window added to the samples in flight when choosing hot rows: unbounded (every
// row hot) when the tables fit in one XCD's L2, where atomics stay on chip and the few rows
// collide constantly; else none (rows are read and written coherently, see tile.hpp).
inline double small_table_window(double l2_bytes, double footprint)
{
    return footprint <= l2_bytes ? __builtin_inf() : 0.0;
}

ScratchLayout scratch_layout(long long n, long long m);

// Bytes of the static build scratch of lh_build_alias_noalloc (per GPU): enough for
// scratch_layout(n, m) with n, m <= 2^21.
constexpr size_t kNoAllocScratchBytes = 65ull << 20;
constexpr long long kNoAllocMaxItems = 1ll << 21;  // largest n and largest m it accepts
// Look up that array's device address on `device` (current) once; lh_create calls it.
hipError_t noalloc_scratch_setup(int device);

constexpr int RADIX_ITEMS = 16;
constexpr int RADIX_THREADS = 256;
constexpr int RADIX_TILE = RADIX_ITEMS * RADIX_THREADS;

}  // namespace lh

struct lh_handle {
    lh_params p{};
    int device = 0;
    int num_cu = 256;
    double l2_bytes = 4194304.0;  // L2 bytes of one XCD
    hipStream_t stream = nullptr;
    bool bound = false, graph_set = false, edge_ready = false, neg_ready = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    void *tab[3] = {nullptr, nullptr, nullptr};
    long long n = 0, m = 0;
    long long n_active = 0;  // nodes with at least one arc (from the last alias build)
    unsigned long long heat_count[256] = {};  // nodes per heat value (last build or import)
    const int32_t *src = nullptr, *dst = nullptr;
    const float *w = nullptr;
    lh::WsLayout lay;
    EdgeRec *erec = nullptr;
    NegRec *nrec = nullptr;
    unsigned int *status = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    lh::TileCfg cfg;  // chosen Hogwild kernel configuration
    bool cfg_pinned = false;  // set by lh_set_kernel_config or lh_tune: auto_cfg leaves it
    lh::WalkState walk;       // random-walk pair source, when one is built
    std::string err;
};

namespace lh {
lh::GraphDev graph_dev(const lh_handle *h);
lh_status fail(lh_handle *h, lh_status s, const std::string &msg);
lh_status hip_fail(lh_handle *h, hipError_t e, const char *what);

// Kernel families (implemented in separate translation units).
lh_status validate_graph(lh_handle *h);
lh_status build_alias(lh_handle *h, void *scratch, size_t bytes);
lh_status import_alias(lh_handle *h, int which, const uint64_t *thr, const int32_t *alias);
lh_status export_alias(lh_handle *h, int which, uint64_t *thr, int32_t *alias);
void launch_init(lh_handle *h);
void launch_sample(lh_handle *h, unsigned long long first, unsigned long long count, int32_t *u,
                   int32_t *v, int32_t *neg, const int2 *pairs = nullptr, unsigned long long pairs_first = 0);
void launch_rw(lh_handle *h, int table, long long row0, long long rows, float *buf, bool write);
TileCfg default_cfg(int dtype, int d);
TileCfg natural_cfg(int dtype, int d);
// Share of row touches (0..1) that fall on rows of heat <= hot_heat, from the per-heat node
// counts: a node of heat v is touched by one sample with probability in [2^-(v+1), 2^-v)
// (2^-(v+1/2) is taken) and a sample touches 2 + K rows of each table.
double hot_touch_share(const unsigned long long *heat_count, int hot_heat, int K);
// Samples in flight of a Hogwild launch of `count` samples in configuration c.
double hogwild_in_flight(const GraphDev &g, int dtype, int orders, const TileCfg &c, unsigned long long count,
                         int num_cu);
// Largest hot share at which a bfloat16 handle runs two samples per wavefront.
constexpr double kTwoPerWaveMaxHotShare = 0.1;
// The Hogwild configuration of a handle none was pinned for, once its degrees are known.
// bfloat16: two samples per wavefront (half the lanes, twice the units per lane) when at
// most kTwoPerWaveMaxHotShare of the row touches then fall on hot rows, else one.  Two per
// wavefront double the samples in flight, which hides more of the latency of random rows
// in large tables, but they also enlarge the hot set, whose atomics cost more than that
// gain where hub rows take a large share of the touches.  Binary32: default_cfg.
TileCfg auto_cfg(const lh_handle *h);
bool cfg_supported(int dtype, int d, const TileCfg &c);
hipError_t launch_hogwild(const GraphDev &g, int dtype, int orders, const TileCfg &c,
                          unsigned long long first, unsigned long long end, int num_cu,
                          const ShadowCtx *sc, hipStream_t s);
// The shadow context of a bfloat16 Hogwild handle (false for other handles).
bool shadow_ctx(const lh_handle *h, ShadowCtx *out);
// Before a launch: trim hot_heat so the hot set fits the shadow, give each hot node a
// slot (others -1) and widen its rows into the shadow.  After: round the shadow rows back
// into the tables (stochastic rounding keyed by `first`).
hipError_t shadow_begin(const ShadowCtx &sc, int hot_heat, hipStream_t s);
hipError_t shadow_end(const ShadowCtx &sc, int hot_heat, unsigned long long first, hipStream_t s);
lh_status train_snapshot(lh_handle *h, unsigned long long first, unsigned long long count,
                         const int2 *pairs = nullptr, unsigned long long pairs_first = 0);
// Walk pair source: for each buffer fill (chunk) that overlaps [first, first + count),
// generate its pairs unless the buffer holds them already, then call
// body(sub_first, sub_count, pairs, pairs_first) for the overlap.
lh_status walk_each_chunk(lh_handle *h, unsigned long long first, unsigned long long count,
                          const std::function<lh_status(unsigned long long, unsigned long long, const int2 *,
                                                        unsigned long long)> &body);
// Stable LSD radix sort of (keys, values) on the low `bits` bits of the keys, 4-bit digits,
// each thread ranking its items in order (so equal keys keep their input order).  ka/va
// hold the input, kb/vb are the other buffers of the ping-pong; *kout/*vout receive the
// buffers that hold the result.  hist: 16 * ceil(E / RADIX_TILE) words; ilev: the scan
// levels of that many words.  E < 2^32.
void radix_sort_u32(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, long long E, int bits, uint32_t *hist,
                    uint32_t *ilev, hipStream_t s, uint32_t **kout, uint32_t **vout);
}  // namespace lh
