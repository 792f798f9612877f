// C ABI of the linehip library: argument checks, handle state, stream ordering.
#include <cmath>
#include <cstring>
#include <new>

#include "handle.hpp"

namespace lh {

lh_status fail(lh_handle *h, lh_status s, const std::string &msg)
{
    if (h) h->err = msg;
    return s;
}

lh_status hip_fail(lh_handle *h, hipError_t e, const char *what)
{
    if (h) h->err = std::string(what) + ": " + hipGetErrorString(e);
    return LH_ERR_HIP;
}

GraphDev graph_dev(const lh_handle *h)
{
    GraphDev g;
    for (int t = 0; t < 3; ++t) g.tab[t] = h->tab[t];
    g.erec = h->erec;
    g.nrec = h->nrec;
    g.m = h->m;
    g.n = h->n;
    g.seed = h->p.seed;
    g.key1 = (unsigned long long)(uint32_t)h->p.graph_id;
    g.sr_key = (2ull << 32) | (unsigned long long)(uint32_t)h->p.graph_id;
    g.T = h->p.total_samples;
    g.eta0 = h->p.eta0;
    g.lambda = (float)h->p.lambda;
    g.alpha = (float)h->p.alpha_neg;
    g.eta_scale = 1.0f;
    g.d = h->p.d;
    g.nunits = h->p.dtype == LH_FP32 ? h->p.d : h->p.d / 2;
    g.K = h->p.K;
    g.hot_heat = -1;
    g.hot_rate = h->p.hot_rate;
    g.max_in_flight = 0.0;
    if (h->p.max_conflicts > 0.0 && h->n_active > 0)
        g.max_in_flight = h->p.max_conflicts * (double)h->n_active / (double)(h->p.K + 2);
    const double b = h->p.dtype == LH_FP32 ? 4.0 : 2.0;
    const double ntab = h->p.orders == LH_ORDER12 ? 3.0 : (h->p.orders == LH_ORDER2 ? 2.0 : 1.0);
    const double rows = (double)(h->n_active > 0 ? h->n_active : h->n);
    g.resid = small_table_window(h->l2_bytes, rows * h->p.d * b * ntab);
    ShadowCtx sc;
    const bool shadowed = shadow_ctx(h, &sc);
    for (int t = 0; t < 3; ++t) g.shadow[t] = shadowed ? sc.shadow[t] : nullptr;
    g.slot = shadowed ? sc.slot : nullptr;
    g.tiles = h->ws ? (unsigned long long *)(h->ws + h->lay.tiles) : nullptr;
    g.pairs = nullptr;
    g.pairs_first = 0;
    g.heat = h->ws ? (const uint8_t *)(h->ws + h->lay.nheat) : nullptr;
    g.pool_n = 0;
    return g;
}

static lh_status check_params(const lh_params *p)
{
    if (!p) return LH_ERR_INVALID_ARG;
    if (p->d < 8 || p->d > 512 || p->d % 8 != 0) return LH_ERR_INVALID_ARG;
    if (p->K < 0 || p->K > 8) return LH_ERR_INVALID_ARG;
    if (p->orders < 1 || p->orders > 3) return LH_ERR_INVALID_ARG;
    if (p->dtype != LH_FP32 && p->dtype != LH_BF16) return LH_ERR_INVALID_ARG;
    if (!std::isfinite(p->eta0) || p->eta0 < 0) return LH_ERR_INVALID_ARG;
    if (!std::isfinite(p->lambda) || p->lambda < 0) return LH_ERR_INVALID_ARG;
    if (!std::isfinite(p->alpha_neg)) return LH_ERR_INVALID_ARG;
    if (std::isnan(p->hot_rate) || std::isnan(p->max_conflicts)) return LH_ERR_INVALID_ARG;
    if (p->hot_shadow != 0 && p->hot_shadow != 1) return LH_ERR_INVALID_ARG;
    if (p->total_samples == 0) return LH_ERR_INVALID_ARG;
    if (p->graph_id < 0) return LH_ERR_INVALID_ARG;
    if (p->mode != LH_HOGWILD && p->mode != LH_SNAPSHOT) return LH_ERR_INVALID_ARG;
    if (p->mode == LH_SNAPSHOT) {
        if (p->batch < 1) return LH_ERR_INVALID_ARG;
        long long nord = p->orders == 3 ? 2 : 1;
        long long E = p->batch * nord * (long long)(p->K + 2);
        if (p->batch > (1ll << 26) || E >= (1ll << 31)) return LH_ERR_INVALID_ARG;
    }
    return LH_OK;
}

static lh_status check_sizes(const lh_params *p, long long n, long long m)
{
    if (n < 1 || n >= (1ll << 31) || m < 0 || m >= (1ll << 31)) return LH_ERR_INVALID_ARG;
    if (p->mode == LH_SNAPSHOT && 3ll * n >= (1ll << 32)) return LH_ERR_INVALID_ARG;
    return LH_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

static bool ready(const lh_handle *h) { return h->bound && h->graph_set && h->edge_ready && h->neg_ready; }

static bool table_used(const lh_handle *h, int t)
{
    if (t == LH_TABLE_U || t == LH_TABLE_C) return (h->p.orders & 2) != 0;
    if (t == LH_TABLE_U1) return (h->p.orders & 1) != 0;
    return false;
}

}  // namespace lh

using namespace lh;

static const char *const kSymbols[] = {
    "lh_create",          "lh_workspace_size", "lh_bind",          "lh_set_graph",       "lh_build_alias",     "lh_build_alias_noalloc",
    "lh_import_alias",    "lh_export_alias",   "lh_init_embeddings", "lh_sample",        "lh_train_steps",
    "lh_read_embeddings", "lh_write_embeddings", "lh_check",       "lh_last_train_ms",   "lh_tune",   "lh_kernel_config", "lh_set_kernel_config",
    "lh_status_string",   "lh_last_error",     "lh_destroy",       "lh_batch_create",    "lh_batch_tune",
    "lh_batch_capture",   "lh_batch_launch",   "lh_batch_run",     "lh_batch_last_ms",   "lh_batch_config",    "lh_batch_done",      "lh_batch_destroy",
    "lh_walk_size",       "lh_walk_build",     "lh_walk_pairs",    "lh_walk_export",     "lh_walk_detach",
    "lh_walk_pool_size",  "lh_walk_pool",
    "lh_abi_symbol_count", "lh_abi_symbol_name",
};

extern "C" {

int lh_abi_symbol_count(void) { return (int)(sizeof(kSymbols) / sizeof(kSymbols[0])); }

const char *lh_abi_symbol_name(int i)
{
    if (i < 0 || i >= lh_abi_symbol_count()) return nullptr;
    return kSymbols[i];
}

const char *lh_status_string(lh_status s)
{
    switch (s) {
    case LH_OK: return "ok";
    case LH_ERR_INVALID_ARG: return "invalid argument";
    case LH_ERR_OUT_OF_RANGE: return "vertex id out of range";
    case LH_ERR_ZERO_WEIGHT: return "invalid or zero total weight";
    case LH_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case LH_ERR_NOT_BUILT: return "not bound, graph not set or alias tables not built";
    case LH_ERR_UNSUPPORTED: return "unsupported parameter combination";
    case LH_ERR_NO_DEVICE: return "no HIP device";
    case LH_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *lh_last_error(const lh_handle *h) { return h ? h->err.c_str() : ""; }

lh_status lh_create(lh_handle **out, const lh_params *p, int device)
{
    if (!out) return LH_ERR_INVALID_ARG;
    *out = nullptr;
    lh_status st = check_params(p);
    if (st != LH_OK) return st;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return LH_ERR_NO_DEVICE;
    }
    if (device < 0 || device >= count) return LH_ERR_NO_DEVICE;
    lh_handle *h = new (std::nothrow) lh_handle();
    if (!h) return LH_ERR_HIP;
    h->p = *p;
    h->device = device;
    DeviceGuard g(device);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        h->num_cu = cus;
    int l2 = 0;
    if (hipDeviceGetAttribute(&l2, hipDeviceAttributeL2CacheSize, device) == hipSuccess && l2 > 0)
        h->l2_bytes = (double)l2;
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
        delete h;
        return LH_ERR_HIP;
    }
    h->cfg = default_cfg(p->dtype, p->d);
    // The static scratch of lh_build_alias_noalloc: its address on this device, looked up
    // once per device here at set-up (a failure is reported by that call, not here).
    (void)noalloc_scratch_setup(device);
    *out = h;
    return LH_OK;
}

lh_status lh_workspace_size(const lh_params *p, int64_t n, int64_t m, size_t *persist, size_t *scratch)
{
    lh_status st = check_params(p);
    if (st != LH_OK) return st;
    if (!persist || !scratch) return LH_ERR_INVALID_ARG;
    st = check_sizes(p, n, m);
    if (st != LH_OK) return st;
    *persist = ws_layout(*p, n, m).total;
    *scratch = scratch_layout(n, m).total;
    return LH_OK;
}

lh_status lh_bind(lh_handle *h, void *workspace, size_t bytes, void *const tables[3], void *stream)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace & 255u) != 0) return fail(h, LH_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (!tables) return fail(h, LH_ERR_INVALID_ARG, "tables is NULL");
    for (int t = 0; t < 3; ++t) {
        if (table_used(h, t) && (!tables[t] || ((uintptr_t)tables[t] & 15u) != 0))
            return fail(h, LH_ERR_INVALID_ARG, "a table the orders use is NULL or not 16-byte aligned");
    }
    h->ws = (char *)workspace;
    h->ws_bytes = bytes;
    for (int t = 0; t < 3; ++t) h->tab[t] = table_used(h, t) ? tables[t] : nullptr;
    h->stream = (hipStream_t)stream;
    h->bound = true;
    h->graph_set = h->edge_ready = h->neg_ready = false;
    h->walk = WalkState();
    return LH_OK;
}

lh_status lh_set_graph(lh_handle *h, int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->bound) return fail(h, LH_ERR_NOT_BUILT, "lh_bind first");
    if (check_sizes(&h->p, n, m) != LH_OK) return fail(h, LH_ERR_INVALID_ARG, "n or m out of range");
    if (m > 0 && (!src || !dst || !w)) return fail(h, LH_ERR_INVALID_ARG, "arc arrays are NULL");
    WsLayout L = ws_layout(h->p, n, m);
    if (h->ws_bytes < L.total) return fail(h, LH_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than lh_workspace_size");
    h->lay = L;
    h->n = n;
    h->m = m;
    h->src = src;
    h->dst = dst;
    h->w = w;
    h->status = (unsigned int *)(h->ws + L.status);
    h->erec = (EdgeRec *)(h->ws + L.erec);
    h->nrec = (NegRec *)(h->ws + L.nrec);
    h->graph_set = false;
    h->edge_ready = h->neg_ready = false;
    h->walk = WalkState();
    DeviceGuard g(h->device);
    lh_status st = validate_graph(h);
    if (st != LH_OK) return st;
    h->graph_set = true;
    return LH_OK;
}

lh_status lh_build_alias(lh_handle *h, void *scratch, size_t scratch_bytes)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->graph_set) return fail(h, LH_ERR_NOT_BUILT, "lh_set_graph first");
    if (h->m < 1) return fail(h, LH_ERR_ZERO_WEIGHT, "the graph has no arcs");
    DeviceGuard g(h->device);
    return build_alias(h, scratch, scratch_bytes);
}

lh_status lh_import_alias(lh_handle *h, int which, const uint64_t *thr, const int32_t *alias)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->graph_set) return fail(h, LH_ERR_NOT_BUILT, "lh_set_graph first");
    if ((which != LH_ALIAS_EDGE && which != LH_ALIAS_NEG) || !thr || !alias)
        return fail(h, LH_ERR_INVALID_ARG, "bad table selector or NULL arrays");
    if (which == LH_ALIAS_EDGE && h->m < 1) return fail(h, LH_ERR_INVALID_ARG, "the graph has no arcs");
    DeviceGuard g(h->device);
    return import_alias(h, which, thr, alias);
}

lh_status lh_export_alias(lh_handle *h, int which, uint64_t *thr, int32_t *alias)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if ((which != LH_ALIAS_EDGE && which != LH_ALIAS_NEG) || !thr || !alias)
        return fail(h, LH_ERR_INVALID_ARG, "bad table selector or NULL arrays");
    if (!h->graph_set || !(which == LH_ALIAS_EDGE ? h->edge_ready : h->neg_ready))
        return fail(h, LH_ERR_NOT_BUILT, "alias table not built");
    DeviceGuard g(h->device);
    return export_alias(h, which, thr, alias);
}

lh_status lh_init_embeddings(lh_handle *h)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->bound || !h->graph_set) return fail(h, LH_ERR_NOT_BUILT, "lh_bind and lh_set_graph first");
    DeviceGuard g(h->device);
    launch_init(h);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LH_OK : hip_fail(h, e, "init");
}

lh_status lh_sample(lh_handle *h, uint64_t first, uint64_t count, int32_t *u, int32_t *v, int32_t *neg)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!ready(h)) return fail(h, LH_ERR_NOT_BUILT, "alias tables not built");
    if (count > 0 && (!u || !v || (h->p.K > 0 && !neg))) return fail(h, LH_ERR_INVALID_ARG, "NULL output");
    if (first + count < first) return fail(h, LH_ERR_INVALID_ARG, "sample range overflows");
    if (count >= (1ull << 40)) return fail(h, LH_ERR_INVALID_ARG, "count too large");
    DeviceGuard g(h->device);
    if (h->walk.ready)
        return walk_each_chunk(h, first, count,
                               [&](unsigned long long sf, unsigned long long sc, const int2 *pairs,
                                   unsigned long long pf) -> lh_status {
                                   const unsigned long long o = sf - first;
                                   launch_sample(h, sf, sc, u + o, v + o, neg ? neg + o * (unsigned long long)h->p.K : nullptr,
                                                 pairs, pf);
                                   hipError_t e = hipGetLastError();
                                   return e == hipSuccess ? LH_OK : hip_fail(h, e, "sample");
                               });
    launch_sample(h, first, count, u, v, neg);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LH_OK : hip_fail(h, e, "sample");
}

lh_status lh_train_steps(lh_handle *h, uint64_t first, uint64_t count)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!ready(h)) return fail(h, LH_ERR_NOT_BUILT, "alias tables not built");
    if (first + count < first || first + count > h->p.total_samples)
        return fail(h, LH_ERR_INVALID_ARG, "samples beyond total_samples");
    if (h->p.mode == LH_SNAPSHOT && first % (uint64_t)h->p.batch != 0)
        return fail(h, LH_ERR_INVALID_ARG, "SNAPSHOT ranges start at a batch boundary");
    h->timed = false;
    if (count == 0) return LH_OK;
    DeviceGuard g(h->device);
    hipError_t e = hipEventRecord(h->ev0, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "event");
    // One pass over [sf, sf + sc) with positive pairs from `pairs` (NULL: arc draws).
    auto pass = [&](unsigned long long sf, unsigned long long sc, const int2 *pairs,
                    unsigned long long pf) -> lh_status {
        if (h->p.mode == LH_HOGWILD) {
            ShadowCtx shc;
            const bool shadowed = shadow_ctx(h, &shc);
            GraphDev gd = graph_dev(h);
            gd.pairs = pairs;
            gd.pairs_first = pf;
            gd.pool_n = pairs ? h->walk.pool : 0;
            hipError_t le = launch_hogwild(gd, h->p.dtype, h->p.orders, h->cfg, sf, sf + sc, h->num_cu,
                                           shadowed ? &shc : nullptr, h->stream);
            return le == hipSuccess ? LH_OK : hip_fail(h, le, "hogwild launch");
        }
        return train_snapshot(h, sf, sc, pairs, pf);
    };
    lh_status st = h->walk.ready ? walk_each_chunk(h, first, count, pass) : pass(first, count, nullptr, 0);
    if (st != LH_OK) return st;
    e = hipEventRecord(h->ev1, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "event");
    h->timed = true;
    return LH_OK;
}

lh_status lh_set_kernel_config(lh_handle *h, const int32_t cfg[3])
{
    if (!h || !cfg) return LH_ERR_INVALID_ARG;
    TileCfg c;
    c.lps = cfg[0];
    c.upl = cfg[1];
    c.blocks_per_cu = cfg[2];
    if (!cfg_supported(h->p.dtype, h->p.d, c))
        return fail(h, LH_ERR_INVALID_ARG, "no kernel for this (lanes, units, workgroups) at this width");
    h->cfg = c;
    h->cfg_pinned = true;
    return LH_OK;
}

lh_status lh_kernel_config(const lh_handle *h, int32_t out[3])
{
    if (!h || !out) return LH_ERR_INVALID_ARG;
    out[0] = h->cfg.lps;
    out[1] = h->cfg.upl;
    out[2] = h->cfg.blocks_per_cu;
    return LH_OK;
}

lh_status lh_last_train_ms(lh_handle *h, double *ms)
{
    if (!h || !ms) return LH_ERR_INVALID_ARG;
    *ms = 0.0;
    if (!h->timed) return LH_OK;
    DeviceGuard g(h->device);
    hipError_t e = hipEventSynchronize(h->ev1);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, h->ev0, h->ev1);
    if (e != hipSuccess) return hip_fail(h, e, "event timing");
    *ms = (double)f;
    return LH_OK;
}

static lh_status rw(lh_handle *h, int table, int64_t row0, int64_t rows, float *buf, bool write)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->bound || !h->graph_set) return fail(h, LH_ERR_NOT_BUILT, "lh_bind and lh_set_graph first");
    if (!table_used(h, table) || !buf || row0 < 0 || rows < 0 || row0 + rows > h->n)
        return fail(h, LH_ERR_INVALID_ARG, "bad table or row range");
    DeviceGuard g(h->device);
    launch_rw(h, table, row0, rows, buf, write);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LH_OK : hip_fail(h, e, "table copy");
}

lh_status lh_read_embeddings(lh_handle *h, int table, int64_t row0, int64_t rows, float *out)
{
    return rw(h, table, row0, rows, out, false);
}

lh_status lh_write_embeddings(lh_handle *h, int table, int64_t row0, int64_t rows, const float *in)
{
    return rw(h, table, row0, rows, const_cast<float *>(in), true);
}

lh_status lh_check(lh_handle *h)
{
    if (!h) return LH_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "stream");
    if (!h->status) return LH_OK;
    unsigned int st = 0;
    e = hipMemcpy(&st, h->status, sizeof(st), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "status read");
    if (st) {
        unsigned int zero = 0;
        e = hipMemcpy(h->status, &zero, sizeof(zero), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(h, e, "status clear");
    }
    if (st & ST_OUT_OF_RANGE) return fail(h, LH_ERR_OUT_OF_RANGE, "an imported alias entry was out of range");
    if (st & (ST_BAD_WEIGHT | ST_ZERO_TOTAL)) return fail(h, LH_ERR_ZERO_WEIGHT, "invalid weights");
    return LH_OK;
}

lh_status lh_destroy(lh_handle *h)
{
    if (!h) return LH_ERR_INVALID_ARG;
    {
        DeviceGuard g(h->device);
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        if (h->ev0) (void)hipEventDestroy(h->ev0);
        if (h->ev1) (void)hipEventDestroy(h->ev1);
    }
    delete h;
    return LH_OK;
}

}  // extern "C"
