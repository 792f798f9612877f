// Autotuning of the Hogwild kernel, and many graphs trained in one persistent launch.
//
// Batched training: every graph's sample range [0, T_g) is cut into items of S samples.
// One persistent kernel is launched with a fixed grid; each wavefront takes the next
// item from a device counter, finds its graph by binary search over the items' prefix
// offsets, trains the item's 64-sample tiles with the per-sample body used by the
// single-graph kernel (a width-specific tile configuration chosen inside the kernel), and
// takes another item until none is left, so every wave reaches the exit.  A counter per
// graph records how many samples were trained.  The reset of the counters (a kernel, not
// a memset) and the persistent kernel are captured into one hipGraph.
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "handle.hpp"
#include "sgd_kernels.hpp"

namespace lh {

// ---------------------------------------------------------------------------
// Tuning cache: a flat JSON object {"key": [lps, cpl, blocks_per_cu, extra], ...}.
// ---------------------------------------------------------------------------
static bool cache_lookup(const char *path, const std::string &key, int out[4])
{
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    std::string s = ss.str();
    std::string pat = "\"" + key + "\": [";
    size_t at = s.find(pat);
    if (at == std::string::npos) return false;
    return std::sscanf(s.c_str() + at + pat.size(), "%d, %d, %d, %d", &out[0], &out[1], &out[2], &out[3]) == 4;
}

static void cache_store(const char *path, const std::string &key, const int v[4])
{
    if (!path) return;
    std::string s;
    {
        std::ifstream f(path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            s = ss.str();
        }
    }
    std::vector<std::string> lines;
    size_t pos = 0;
    while (true) {  // keep existing entries other than this key
        size_t q0 = s.find('"', pos);
        if (q0 == std::string::npos) break;
        size_t q1 = s.find('"', q0 + 1);
        size_t b1 = s.find(']', q1);
        if (q1 == std::string::npos || b1 == std::string::npos) break;
        std::string k = s.substr(q0 + 1, q1 - q0 - 1);
        if (k != key) lines.push_back(s.substr(q0, b1 - q0 + 1));
        pos = b1 + 1;
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf), "\"%s\": [%d, %d, %d, %d]", key.c_str(), v[0], v[1], v[2], v[3]);
    lines.push_back(buf);
    std::ofstream o(path);
    o << "{\n";
    for (size_t i = 0; i < lines.size(); ++i) o << "  " << lines[i] << (i + 1 < lines.size() ? ",\n" : "\n");
    o << "}\n";
}

static std::string arch_name(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

static int log2_bucket(long long x)
{
    int b = 0;
    while ((1ll << (b + 1)) <= x) ++b;
    return b;
}

}  // namespace lh

using namespace lh;

extern "C" lh_status lh_tune(lh_handle *h, uint64_t probe, const char *cache_path)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->bound || !h->graph_set || !h->edge_ready || !h->neg_ready)
        return fail(h, LH_ERR_NOT_BUILT, "alias tables not built");
    if (h->p.mode != LH_HOGWILD) return LH_OK;
    if (probe < 64 || probe > h->p.total_samples) return fail(h, LH_ERR_INVALID_ARG, "probe out of range");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != h->device) (void)hipSetDevice(h->device);
    char key[160];
    std::snprintf(key, sizeof(key), "%s|hogwild-upl|dt%d|d%d|K%d|o%d|n%d", arch_name(h->device).c_str(), h->p.dtype,
                  h->p.d, h->p.K, h->p.orders, log2_bucket(h->n));
    int hit[4];
    if (cache_lookup(cache_path, key, hit)) {
        TileCfg c;
        c.lps = hit[0];
        c.upl = hit[1];
        c.blocks_per_cu = hit[2];
        if (cfg_supported(h->p.dtype, h->p.d, c)) {
            h->cfg = c;
            h->cfg_pinned = true;
            return LH_OK;
        }
    }
    const int nu = h->p.dtype == LH_FP32 ? h->p.d : h->p.d / 2;
    GraphDev g = graph_dev(h);
    // Dry run: the step size is scaled to zero, so every row is written back unchanged,
    // and hot rows still issue their atomics (bfloat16 ones too, whose zero increments the
    // masked training kernels skip), so the timing includes what the hot set costs.
    g.eta_scale = 0.0f;
    const int bpc_opts[] = {1, 2, 3, 4, 8, 16};
    // Candidate shapes: the compiled (lanes, units) that cover a row with the fewest
    // 4-byte slots (wider groups would only idle lanes).
    std::vector<TileCfg> shapes;
    int cover = 1 << 30;
#define LH_TUNE_COVER(L, U) \
    if (L * U >= nu && L * U < cover) cover = L * U;
    LH_CFG_LIST(LH_TUNE_COVER)
#undef LH_TUNE_COVER
#define LH_TUNE_SHAPE(L, U)      \
    if (L * U == cover) {        \
        TileCfg c;               \
        c.lps = L;               \
        c.upl = U;               \
        shapes.push_back(c);     \
    }
    LH_CFG_LIST(LH_TUNE_SHAPE)
#undef LH_TUNE_SHAPE
    TileCfg best = h->cfg;
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LH_ERR_HIP;
    for (TileCfg c : shapes) {
        for (int bpc : bpc_opts) {
            c.blocks_per_cu = bpc;
            if (!cfg_supported(h->p.dtype, h->p.d, c)) continue;
            // warm-up, then timed
            hipError_t er = launch_hogwild(g, h->p.dtype, h->p.orders, c, 0, probe / 4, h->num_cu, nullptr,
                                           h->stream);
            if (er != hipSuccess) continue;
            (void)hipEventRecord(e0, h->stream);
            (void)launch_hogwild(g, h->p.dtype, h->p.orders, c, 0, probe, h->num_cu, nullptr, h->stream);
            (void)hipEventRecord(e1, h->stream);
            if (hipEventSynchronize(e1) != hipSuccess) continue;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->cfg = best;
    h->cfg_pinned = true;
    int v[4] = {best.lps, best.upl, best.blocks_per_cu, 0};
    cache_store(cache_path, key, v);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LH_OK : hip_fail(h, e, "tune");
}

// ===========================================================================
// Batched persistent training.
// ===========================================================================
namespace lh {

struct BatchDesc {
    GraphDev g;
    unsigned long long item0;  // index of this graph's first item
    unsigned long long limit;  // samples to train: [0, limit)
};

// The work queue hands out items in the order of sched: item i trains chunk
// (sched[i] & (2^40 - 1)) of graph (sched[i] >> 40).  The host interleaves every graph's
// chunks in proportion to its size, so at any moment the wavefronts in flight are spread
// over the graphs by size and no small graph receives the whole GPU at once (which would
// put thousands of concurrent writers on each of its rows).
struct BatchArgs {
    const BatchDesc *desc;
    const unsigned long long *sched;
    int G;
    unsigned long long total_items;
    unsigned long long item_samples;
    unsigned long long *queue;
    unsigned long long *done;  // [G]
};

// Tile configurations by variant (lanes per sample, units per lane).  Binary32: 0 = four
// units per lane, 1 = half the lanes with eight units each.  bfloat16: 0 = one unit per
// lane (the fastest single-graph shape), 1 = four units per lane.  The small tile serves
// rows of at most LS * US units, the large one the rest.
template <typename TT, int V>
struct BatchCfg;
template <>
struct BatchCfg<uint16_t, 0> {
    static constexpr int LS = 32, US = 1, LL = 64, UL = 1;
};
template <>
struct BatchCfg<uint16_t, 1> {
    static constexpr int LS = 8, US = 4, LL = 16, UL = 4;
};
template <>
struct BatchCfg<float, 0> {
    static constexpr int LS = 16, US = 4, LL = 32, UL = 4;
};
template <>
struct BatchCfg<float, 1> {
    static constexpr int LS = 8, US = 8, LL = 16, UL = 8;
};

__global__ void k_batch_reset(unsigned long long *queue, unsigned long long *done, int G)
{
    int i = threadIdx.x;
    if (i == 0) queue[0] = 0ull;
    for (int g = i; g < G; g += blockDim.x) done[g] = 0ull;
}

// Register budget of the batched kernel (it holds two tile shapes): at least 3 waves per
// SIMD, or 4 for bfloat16 with the shadow path.  Measured on C4 (bfloat16): without the
// shadow path 3 waves (no spills) ran 1,785 M samples/s against 1,124 M at 4 waves (with
// spills); with the path 4 waves ran 1,262 M against 1,084 M at 3 and 990 M at 5.
template <typename TT, bool SH>
constexpr int batch_min_waves() { return sizeof(TT) == 2 && SH ? 4 : 3; }

// SH: the shadow path is compiled in (a graph may keep its hot rows in a binary32 shadow).
template <typename TT, int KMAX, int V, bool SH>
__global__ void __launch_bounds__(256, (batch_min_waves<TT, SH>())) k_batch(BatchArgs a)
{
    using Cfg = BatchCfg<TT, V>;
    const int lane = threadIdx.x & 63;
    SnapOut so{};
    while (true) {
        unsigned long long item = 0;
        if (lane == 0) item = atomicAdd(a.queue, 1ull);
        item = ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(item >> 32)) << 32) |
               (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(item & 0xffffffffull));
        if (item >= a.total_items) break;
        const unsigned long long packed = a.sched[item];
        const int lo = (int)(packed >> 40);
        const unsigned long long chunk = packed & ((1ull << 40) - 1);
        const BatchDesc &D = a.desc[lo];
        const GraphDev g = D.g;
        unsigned long long s0 = chunk * a.item_samples;
        unsigned long long s1 = s0 + a.item_samples;
        if (s1 > D.limit) s1 = D.limit;
        // rows that one of the two tiles covers exactly take it without bounds masks (graphs
        // with KMAX negatives)
        const bool kfull = g.K == KMAX;
        if (kfull && g.nunits == Cfg::LS * Cfg::US) {
            for (unsigned long long t = s0; t < s1; t += 64)
                sgd_tile<TT, Cfg::LS, Cfg::US, KMAX, 2, false, SH, true>(g, t, s1, so);
        } else if (kfull && g.nunits == Cfg::LL * Cfg::UL) {
            for (unsigned long long t = s0; t < s1; t += 64)
                sgd_tile<TT, Cfg::LL, Cfg::UL, KMAX, 2, false, SH, true>(g, t, s1, so);
        } else {
            for (unsigned long long t = s0; t < s1; t += 64)
                sgd_tile<TT, Cfg::LL, Cfg::UL, KMAX, 2, false, SH>(g, t, s1, so);
        }
        if (lane == 0 && s1 > s0) atomicAdd(&a.done[lo], s1 - s0);
    }
}

}  // namespace lh

struct lh_batch {
    std::vector<lh_handle *> hs;
    int G = 0;
    int dtype = 0, K = 0, device = 0, num_cu = 256;
    hipStream_t stream = nullptr;
    lh::BatchDesc *d_desc = nullptr;        // device, owned
    unsigned long long *d_ctr = nullptr;    // device, owned: [0] queue, [1..G] done
    unsigned long long *d_sched = nullptr;  // device, owned: item schedule (sched_cap entries)
    size_t sched_cap = 0;
    std::vector<lh::BatchDesc> desc;
    std::vector<unsigned long long> sched;
    int variant = 0, blocks_per_cu = 8;
    unsigned grid = 1;  // blocks of the persistent kernel (set with the schedule)
    unsigned long long item_samples = 8192;
    unsigned long long total_items = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t join0 = nullptr, join1 = nullptr;  // ordering against a caller's stream
    bool timed = false;
};

namespace lh {

// Resident blocks per CU and lanes per sample of the narrower tile configuration of a
// batched kernel variant (the narrower one gives the upper bound on samples in flight, so
// hot rows are over- rather than under-counted).
// Whether some graph of the batch keeps its hot rows in a binary32 shadow: then the kernel
// built with the shadow path runs (it checks per graph whether a shadow is in use).
static bool batch_shadow(const lh_batch *b)
{
    for (const lh_handle *h : b->hs)
        if (uses_shadow(h->p)) return true;
    return false;
}


static int batch_occupancy(const lh_batch *b, int variant, int *ls_out)
{
    int occ = 0, ls = 8;
    const bool k5 = b->K <= 5, sh = batch_shadow(b);
#define LH_OCC(TT, KM, V, SH)                                                                   \
    {                                                                                           \
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch<TT, KM, V, SH>, 256, 0); \
        ls = BatchCfg<TT, V>::LS;                                                               \
    }
#define LH_OCC_BF(KM, V) { if (sh) LH_OCC(uint16_t, KM, V, true) else LH_OCC(uint16_t, KM, V, false) }
    if (b->dtype == LH_BF16) {
        if (k5) { if (variant == 0) LH_OCC_BF(5, 0) else LH_OCC_BF(5, 1) }
        else { if (variant == 0) LH_OCC_BF(8, 0) else LH_OCC_BF(8, 1) }
    } else {
        if (k5) { if (variant == 0) LH_OCC(float, 5, 0, false) else LH_OCC(float, 5, 1, false) }
        else { if (variant == 0) LH_OCC(float, 8, 0, false) else LH_OCC(float, 8, 1, false) }
    }
#undef LH_OCC_BF
#undef LH_OCC
    *ls_out = ls;
    return occ < 1 ? 8 : occ;
}

// The schedule of a batched launch, its grid and each graph's heat threshold.  Graph g
// holds the share phi_g = T_g / sum T of the samples in flight (the schedule interleaves
// the graphs in proportion), so the grid is lowered until phi_g F stays within every
// graph's staleness cap.  A graph whose tables fit in one L2 has all rows hot, as when
// it is trained alone.
static void batch_items(lh_batch *b, unsigned long long item_samples, bool dry, unsigned long long probe)
{
    unsigned long long acc = 0, total = 0;
    for (int i = 0; i < b->G; ++i) {
        BatchDesc &D = b->desc[i];
        D.g = graph_dev(b->hs[i]);
        D.limit = dry ? (probe < D.g.T ? probe : D.g.T) : D.g.T;
        total += D.limit;
    }
    int ls = 8;
    const int occ = batch_occupancy(b, b->variant, &ls);
    const double per_block = 4.0 * (64.0 / ls);
    double grid = (double)b->num_cu * b->blocks_per_cu;
    for (int i = 0; i < b->G; ++i) {
        const double phi = total ? (double)b->desc[i].limit / (double)total : 0.0;
        const double cap = b->desc[i].g.max_in_flight;
        if (cap > 0.0 && phi > 0.0) grid = std::min(grid, std::max(1.0, std::floor(cap / phi / per_block)));
    }
    b->grid = (unsigned)std::max(1.0, grid);
    const double F = std::min((double)b->grid, (double)b->num_cu * occ) * per_block;
    // (position in [0, 1), graph, chunk): chunk i of a graph with c chunks sits at (i + 1/2) / c.
    std::vector<std::pair<double, unsigned long long>> order;
    for (int i = 0; i < b->G; ++i) {
        BatchDesc &D = b->desc[i];
        const double phi = total ? (double)D.limit / (double)total : 0.0;
        D.g.hot_heat = hot_heat_for(phi * F + D.g.resid, D.g.hot_rate);
        D.g.max_in_flight = 0.0;
        D.g.eta_scale = dry ? 0.0f : 1.0f;
        D.item0 = acc;
        const unsigned long long c = (D.limit + item_samples - 1) / item_samples;
        for (unsigned long long k = 0; k < c; ++k)
            order.emplace_back(((double)k + 0.5) / (double)c, ((unsigned long long)i << 40) | k);
        acc += c;
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, unsigned long long> &x, const std::pair<double, unsigned long long> &y) {
                         return x.first < y.first;
                     });
    b->sched.resize(order.size());
    for (size_t i = 0; i < order.size(); ++i) b->sched[i] = order[i].second;
    b->total_items = acc;
}

static hipError_t batch_launch_raw(lh_batch *b, int variant, int bpc, unsigned long long item_samples,
                                   hipStream_t s)
{
    BatchArgs a;
    a.desc = b->d_desc;
    a.sched = b->d_sched;
    a.G = b->G;
    a.total_items = b->total_items;
    a.item_samples = item_samples;
    a.queue = b->d_ctr;
    a.done = b->d_ctr + 1;
    // bfloat16 graphs with a shadow: their hot rows move into it for the launch.
    for (int i = 0; i < b->G; ++i) {
        ShadowCtx sc;
        if (shadow_ctx(b->hs[i], &sc)) {
            hipError_t e = shadow_begin(sc, b->desc[i].g.hot_heat, s);
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, s, a.queue, a.done, b->G);
    (void)bpc;
    dim3 grid(b->grid), block(256);
    const bool k5 = b->K <= 5, sh = batch_shadow(b);
#define LH_BL(TT, KM, V, SH) hipLaunchKernelGGL((k_batch<TT, KM, V, SH>), grid, block, 0, s, a)
#define LH_BL_BF(KM, V) { if (sh) LH_BL(uint16_t, KM, V, true); else LH_BL(uint16_t, KM, V, false); }
    if (b->dtype == LH_BF16) {
        if (k5) {
            if (variant == 0) LH_BL_BF(5, 0) else LH_BL_BF(5, 1)
        } else {
            if (variant == 0) LH_BL_BF(8, 0) else LH_BL_BF(8, 1)
        }
    } else {
        if (k5) {
            if (variant == 0) LH_BL(float, 5, 0, false); else LH_BL(float, 5, 1, false);
        } else {
            if (variant == 0) LH_BL(float, 8, 0, false); else LH_BL(float, 8, 1, false);
        }
    }
#undef LH_BL_BF
#undef LH_BL
    hipError_t e = hipGetLastError();
    for (int i = 0; i < b->G && e == hipSuccess; ++i) {
        ShadowCtx sc;
        if (shadow_ctx(b->hs[i], &sc)) e = shadow_end(sc, b->desc[i].g.hot_heat, 0, s);
    }
    return e;
}

static hipError_t upload_desc(lh_batch *b)
{
    if (b->sched.size() > b->sched_cap) return hipErrorInvalidValue;
    hipError_t e = hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(BatchDesc) * b->desc.size(),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !b->sched.empty())
        e = hipMemcpyAsync(b->d_sched, b->sched.data(), sizeof(unsigned long long) * b->sched.size(),
                           hipMemcpyHostToDevice, b->stream);
    return e;
}

// The stream a launch or run goes on (NULL: the first handle's stream).  Another stream
// first waits for the work queued on the handles' stream.
static hipStream_t enter_stream(lh_batch *b, void *stream)
{
    hipStream_t s = stream ? (hipStream_t)stream : b->stream;
    if (s != b->stream) {
        (void)hipEventRecord(b->join0, b->stream);
        (void)hipStreamWaitEvent(s, b->join0, 0);
    }
    return s;
}

// After the launch: the handles' stream waits for it, so their later calls see its result.
static hipError_t leave_stream(lh_batch *b, hipStream_t s)
{
    if (s == b->stream) return hipSuccess;
    hipError_t e = hipEventRecord(b->join1, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->join1, 0);
    return e;
}

static void drop_graph(lh_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace lh

extern "C" {

lh_status lh_batch_create(lh_batch **out, int G, lh_handle *const *graphs)
{
    if (!out) return LH_ERR_INVALID_ARG;
    *out = nullptr;
    if (G < 1 || !graphs) return LH_ERR_INVALID_ARG;
    for (int i = 0; i < G; ++i) {
        lh_handle *h = graphs[i];
        if (!h) return LH_ERR_INVALID_ARG;
        if (!h->bound || !h->graph_set || !h->edge_ready || !h->neg_ready) return LH_ERR_NOT_BUILT;
        if (h->p.mode != LH_HOGWILD || h->p.orders != LH_ORDER2) return LH_ERR_UNSUPPORTED;
        if (h->walk.ready) return LH_ERR_UNSUPPORTED;  // the batched kernel draws arcs only
        if (h->p.dtype != graphs[0]->p.dtype || h->device != graphs[0]->device) return LH_ERR_UNSUPPORTED;
        if ((h->p.K <= 5) != (graphs[0]->p.K <= 5)) return LH_ERR_UNSUPPORTED;
        const int nu = h->p.dtype == LH_FP32 ? h->p.d : h->p.d / 2;  // 4-byte units per row
        if (nu > (h->p.dtype == LH_FP32 ? 128 : 64)) return LH_ERR_UNSUPPORTED;
    }
    lh_batch *b = new (std::nothrow) lh_batch();
    if (!b) return LH_ERR_HIP;
    b->hs.assign(graphs, graphs + G);
    b->G = G;
    b->dtype = graphs[0]->p.dtype;
    int kmax = 0;
    for (int i = 0; i < G; ++i) kmax = graphs[i]->p.K > kmax ? graphs[i]->p.K : kmax;
    b->K = kmax;
    b->device = graphs[0]->device;
    b->num_cu = graphs[0]->num_cu;
    b->stream = graphs[0]->stream;
    b->desc.resize(G);
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != b->device) (void)hipSetDevice(b->device);
    // room for the schedule at the smallest item size the tuner tries (2048 samples)
    b->sched_cap = 0;
    for (int i = 0; i < G; ++i) b->sched_cap += (size_t)((graphs[i]->p.total_samples + 2047) / 2048);
    if (hipMalloc(&b->d_desc, sizeof(BatchDesc) * G) != hipSuccess ||
        hipMalloc(&b->d_sched, sizeof(unsigned long long) * (b->sched_cap + 1)) != hipSuccess ||
        hipMalloc(&b->d_ctr, sizeof(unsigned long long) * (G + 1)) != hipSuccess ||
        hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&b->join0, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join1, hipEventDisableTiming) != hipSuccess) {
        lh_batch_destroy(b);
        return LH_ERR_HIP;
    }
    batch_items(b, b->item_samples, false, 0);
    if (upload_desc(b) != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess) {
        lh_batch_destroy(b);
        return LH_ERR_HIP;
    }
    *out = b;
    return LH_OK;
}

lh_status lh_batch_tune(lh_batch *b, const char *cache_path)
{
    if (!b) return LH_ERR_INVALID_ARG;
    char key[160];
    unsigned long long tot = 0;
    for (auto *h : b->hs) tot += h->p.total_samples;
    std::snprintf(key, sizeof(key), "%s|batch|dt%d|K%d|G%d|T%d", arch_name(b->device).c_str(), b->dtype, b->K, b->G,
                  log2_bucket((long long)tot));
    int hit[4];
    if (cache_lookup(cache_path, key, hit) && (hit[0] == 0 || hit[0] == 1) && hit[1] >= 1 && hit[1] <= 64 &&
        hit[2] >= 2048) {
        b->variant = hit[0];
        b->blocks_per_cu = hit[1];
        b->item_samples = (unsigned long long)hit[2];
        drop_graph(b);
        return LH_OK;
    }
    // Dry runs on the first samples of every graph (step size scaled to zero).
    unsigned long long probe = 0;
    for (auto *h : b->hs) probe += h->p.total_samples;
    probe = probe / (unsigned long long)b->G / 50 + 4096;
    const int bpcs[] = {4, 8, 16};
    const unsigned long long items[] = {2048, 8192, 32768};
    float best = 1e30f;
    int bv = b->variant, bb = b->blocks_per_cu;
    unsigned long long bi = b->item_samples;
    for (int v = 0; v < 2; ++v)
        for (int bpc : bpcs)
            for (unsigned long long is : items) {
                b->variant = v;
                b->blocks_per_cu = bpc;
                batch_items(b, is, true, probe);
                if (upload_desc(b) != hipSuccess) return LH_ERR_HIP;
                if (batch_launch_raw(b, v, bpc, is, b->stream) != hipSuccess) return LH_ERR_HIP;  // warm-up
                (void)hipEventRecord(b->ev0, b->stream);
                (void)batch_launch_raw(b, v, bpc, is, b->stream);
                (void)hipEventRecord(b->ev1, b->stream);
                if (hipEventSynchronize(b->ev1) != hipSuccess) return LH_ERR_HIP;
                float ms = 0;
                (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
                if (ms < best) {
                    best = ms;
                    bv = v;
                    bb = bpc;
                    bi = is;
                }
            }
    b->variant = bv;
    b->blocks_per_cu = bb;
    b->item_samples = bi;
    batch_items(b, b->item_samples, false, 0);
    if (upload_desc(b) != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess) return LH_ERR_HIP;
    drop_graph(b);
    int v4[4] = {bv, bb, (int)bi, 0};
    cache_store(cache_path, key, v4);
    return LH_OK;
}

lh_status lh_batch_capture(lh_batch *b)
{
    if (!b) return LH_ERR_INVALID_ARG;
    drop_graph(b);
    batch_items(b, b->item_samples, false, 0);
    if (upload_desc(b) != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess) return LH_ERR_HIP;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return LH_ERR_HIP;
    hipError_t e = batch_launch_raw(b, b->variant, b->blocks_per_cu, b->item_samples, b->stream);
    hipError_t e2 = hipStreamEndCapture(b->stream, &b->graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        drop_graph(b);
        return LH_ERR_HIP;
    }
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
        drop_graph(b);
        return LH_ERR_HIP;
    }
    return LH_OK;
}

lh_status lh_batch_launch(lh_batch *b, void *stream)
{
    if (!b) return LH_ERR_INVALID_ARG;
    if (!b->exec) return LH_ERR_NOT_BUILT;
    hipStream_t s = enter_stream(b, stream);
    (void)hipEventRecord(b->ev0, s);
    if (hipGraphLaunch(b->exec, s) != hipSuccess) return LH_ERR_HIP;
    (void)hipEventRecord(b->ev1, s);
    b->timed = true;
    return leave_stream(b, s) == hipSuccess ? LH_OK : LH_ERR_HIP;
}

lh_status lh_batch_run(lh_batch *b, void *stream)
{
    if (!b) return LH_ERR_INVALID_ARG;
    batch_items(b, b->item_samples, false, 0);
    if (upload_desc(b) != hipSuccess) return LH_ERR_HIP;
    hipStream_t s = enter_stream(b, stream);
    (void)hipEventRecord(b->ev0, s);
    if (batch_launch_raw(b, b->variant, b->blocks_per_cu, b->item_samples, s) != hipSuccess) return LH_ERR_HIP;
    (void)hipEventRecord(b->ev1, s);
    b->timed = true;
    return leave_stream(b, s) == hipSuccess ? LH_OK : LH_ERR_HIP;
}

lh_status lh_batch_last_ms(lh_batch *b, double *ms)
{
    if (!b || !ms) return LH_ERR_INVALID_ARG;
    *ms = 0;
    if (!b->timed) return LH_OK;
    if (hipEventSynchronize(b->ev1) != hipSuccess) return LH_ERR_HIP;
    float f = 0;
    if (hipEventElapsedTime(&f, b->ev0, b->ev1) != hipSuccess) return LH_ERR_HIP;
    *ms = f;
    return LH_OK;
}

lh_status lh_batch_config(const lh_batch *b, int64_t out[3])
{
    if (!b || !out) return LH_ERR_INVALID_ARG;
    out[0] = b->variant;
    out[1] = b->blocks_per_cu;
    out[2] = (int64_t)b->item_samples;
    return LH_OK;
}

lh_status lh_batch_done(lh_batch *b, uint64_t *done_per_graph)
{
    if (!b || !done_per_graph) return LH_ERR_INVALID_ARG;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return LH_ERR_HIP;
    if (hipMemcpy(done_per_graph, b->d_ctr + 1, sizeof(unsigned long long) * b->G, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return LH_ERR_HIP;
    return LH_OK;
}

lh_status lh_batch_destroy(lh_batch *b)
{
    if (!b) return LH_ERR_INVALID_ARG;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_sched) (void)hipFree(b->d_sched);
    if (b->d_ctr) (void)hipFree(b->d_ctr);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->join0) (void)hipEventDestroy(b->join0);
    if (b->join1) (void)hipEventDestroy(b->join1);
    delete b;
    return LH_OK;
}

}  // extern "C"
