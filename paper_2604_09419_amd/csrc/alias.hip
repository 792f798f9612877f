// Graph validation and alias-table construction (binary64, built with -ffp-contract=off).
//
// The two discrete distributions of the method are encoded as alias tables (Walker
// 1977 / Vose 1991): the edge distribution of Algorithm 3's root-edge selection
// (weights w over arcs) and the negative distribution of Eq. (1) (weights
// out-degree^0.75 over nodes).  The construction is the closed form of the sweeping
// construction (Huebschle-Schneider and Sanders, "Parallel Weighted Random Sampling"):
//   W = last element of the canonical scan of w; q_i = fl(fl(w_i N) / W)
//   lights L = {q < 1}, heavies H = {q >= 1}, each in index order
//   D = monotone canonical scan of (1 - q) over L, X = the same of (q - 1) over H
//   light a (start S_a = D[a-1], S_0 = 0): prob q, alias H[min(#{X[k] <= S_a}, |H|-1)]
//   heavy k < |H|-1: j = #{S_a < X[k]} - 1, overflow o = D[j] - X[k] (0 when j < 0,
//   clamped at 0); o > 0 gives prob max(0, 1 - o), alias H[k+1]; else prob 1, self
//   last heavy, or every item when H is empty: prob 1, self
//   thr = prob >= 1 ? 2^64 - 1 : (uint64)(prob 2^64)
// Every step is a single correctly rounded binary64 operation in a fixed order, so
// the tables are bitwise reproducible.
#include <mutex>
#include <vector>

#include "handle.hpp"
#include "scan.hpp"

#pragma clang fp contract(off)

// Build scratch of lh_build_alias_noalloc, for callers that cannot allocate: one array
// per GPU, held from the library's load to the end of the process.  Host code never uses
// this name as an address (in host code it names a host-side stand-in); it uses the
// device address hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) unsigned char scratch[lh::kNoAllocScratchBytes];

namespace lh {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

// Once per device, with that device current: the device address of `scratch` there.
hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_err[device];
}

static void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_done[device] ? g_scratch_ptr[device] : nullptr;
}

// ---------------------------------------------------------------------------
// Validation of the arcs: endpoints in [0, n), weights finite and >= 0.
// ---------------------------------------------------------------------------
__global__ void k_validate(const int32_t *src, const int32_t *dst, const float *w, long long m,
                           long long n, unsigned int *status)
{
    long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= m) return;
    int32_t s = src[a], t = dst[a];
    float x = w[a];
    unsigned int f = 0;
    if (s < 0 || (long long)s >= n || t < 0 || (long long)t >= n) f |= ST_OUT_OF_RANGE;
    if (!(x >= 0.0f) || isinf(x)) f |= ST_BAD_WEIGHT;
    if (f) atomicOr(status, f);
}

__global__ void k_clear_status(unsigned int *status) { status[0] = 0u; }

lh_status validate_graph(lh_handle *h)
{
    hipStream_t s = h->stream;
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, h->status);
    if (h->m > 0)
        hipLaunchKernelGGL(k_validate, dim3((unsigned)LH_CDIV(h->m, 256)), dim3(256), 0, s, h->src,
                           h->dst, h->w, h->m, h->n, h->status);
    unsigned int st = 0;
    hipError_t e = hipMemcpyAsync(&st, h->status, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "graph validation");
    if (st & ST_OUT_OF_RANGE) return fail(h, LH_ERR_OUT_OF_RANGE, "an arc endpoint is outside [0, n)");
    if (st & ST_BAD_WEIGHT) return fail(h, LH_ERR_ZERO_WEIGHT, "a weight is negative, NaN or infinite");
    return LH_OK;
}

// ---------------------------------------------------------------------------
// Weights of the two tables, binary64.
// ---------------------------------------------------------------------------
// Out-degrees add one per run of equal consecutive sources inside a wavefront (arc lists
// are often grouped by source), in-degrees one per arc.  The valid lanes of a wavefront are a
// prefix of it (a = block * 256 + thread), so a run ends at the next run head or at the
// first invalid lane.
__global__ void __launch_bounds__(256) k_degrees(const int32_t *src, const int32_t *dst, long long m, int32_t *deg,
                                                 int32_t *indeg)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = a < m;
    const int s = ok ? src[a] : -1;
    if (ok) atomicAdd(&indeg[dst[a]], 1);
    const int lane = (int)(threadIdx.x & 63u);
    const int prev = __shfl_up(s, 1);
    const bool head = ok && (lane == 0 || prev != s);
    const unsigned long long heads = __ballot(head);
    const int nvalid = __popcll(__ballot(ok));
    if (head) {
        const unsigned long long above = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
        int next = above ? __ffsll((long long)above) - 1 : 64;
        if (next > nvalid) next = nvalid;
        atomicAdd(&deg[s], next - lane);
    }
}

// Heat of node r (see common.hpp): floor(-log2 p_r), p_r = (out + in) / m + K nu_r / W_nu.
// It only chooses between the write paths of the training kernel, so it is computed in
// ordinary binary64 arithmetic.  cnt[0] counts the nodes with an arc, cnt[1 + h] the
// nodes of heat h (a per-block histogram in LDS, then one atomic per bin).  256 threads.
__global__ void __launch_bounds__(256) k_heat(const int32_t *deg, const int32_t *indeg, const double *nu,
                                              const double *nu_scan, long long n, long long m, int K, uint8_t *heat,
                                              unsigned long long *cnt)
{
    __shared__ unsigned int hist[256];
    __shared__ unsigned int active;
    hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) active = 0u;
    __syncthreads();
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) {
        if (deg[r] + indeg[r] > 0) atomicAdd(&active, 1u);
        const double Wn = nu_scan[n - 1];
        double p = (double)(deg[r] + indeg[r]) / (double)m;
        if (Wn > 0.0) p += (double)K * nu[r] / Wn;
        int hv = 255;
        if (p > 0.0) {
            const double t = floor(-log2(p));
            hv = t < 0.0 ? 0 : (t > 254.0 ? 254 : (int)t);
        }
        heat[r] = (uint8_t)hv;
        atomicAdd(&hist[hv], 1u);
    }
    __syncthreads();
    if (hist[threadIdx.x]) atomicAdd(&cnt[1 + threadIdx.x], (unsigned long long)hist[threadIdx.x]);
    if (threadIdx.x == 0 && active) atomicAdd(&cnt[0], (unsigned long long)active);
}

__global__ void k_zero_i32(int32_t *p, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_zero_u64(unsigned long long *p, int count)
{
    if ((int)threadIdx.x < count) p[threadIdx.x] = 0ull;
}

__global__ void k_fill_u8(uint8_t *p, long long n, uint8_t v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_edge_weights(const float *w, long long m, double *wq)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) wq[i] = (double)w[i];
}

// Eq. (1) numerator: d^0.75 = sqrt(d) * sqrt(sqrt(d)), each step correctly rounded.
__global__ void k_neg_weights(const int32_t *deg, long long n, double *wq)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = __dsqrt_rn((double)deg[i]);
    double t = __dsqrt_rn(s);
    wq[i] = __dmul_rn(s, t);
}

// q_i = fl(fl(w_i N) / W) in place; light flag (q < 1) into lpos.  A total that is not a
// positive finite number flags ST_ZERO_TOTAL and makes every item heavy (prob 1, self).
__global__ void k_normalise(double *wq, const double *scan, long long N, int32_t *lpos,
                            unsigned int *status)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double W = scan[N - 1];
    bool ok = W > 0.0 && !isinf(W);
    double q = ok ? __ddiv_rn(__dmul_rn(wq[i], (double)N), W) : 1.0;
    if (!ok && i == 0) atomicOr(status, ST_ZERO_TOTAL);
    wq[i] = q;
    lpos[i] = q < 1.0 ? 1 : 0;
}

// Split into lights (prefix of dx/idx) and heavies (suffix), each in index order.
__global__ void k_split(const double *q, const int32_t *lincl, long long N, long long nL, double *dx,
                        int32_t *idx)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double qi = q[i];
    long long inc = lincl[i];
    if (qi < 1.0) {
        long long a = inc - 1;
        dx[a] = __dsub_rn(1.0, qi);
        idx[a] = (int32_t)i;
    } else {
        long long k = i - inc;
        dx[nL + k] = __dsub_rn(qi, 1.0);
        idx[nL + k] = (int32_t)i;
    }
}

__device__ __forceinline__ unsigned long long prob_to_thr(double prob)
{
    if (prob >= 1.0) return ~0ull;
    return (unsigned long long)__dmul_rn(prob, 18446744073709551616.0);
}

// #{k : X[k] <= s}
__device__ __forceinline__ long long count_le(const double *X, long long nH, double s)
{
    long long lo = 0, hi = nH;
    while (lo < hi) {
        long long mid = lo + (hi - lo) / 2;
        if (X[mid] <= s)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// #{a : S_a < x} with S_0 = 0 and S_a = D[a-1]
__device__ __forceinline__ long long count_start_lt(const double *D, long long nL, double x)
{
    if (nL == 0 || !(0.0 < x)) return 0;
    long long lo = 0, hi = nL - 1;
    while (lo < hi) {
        long long mid = lo + (hi - lo) / 2;
        if (D[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return 1 + lo;
}

struct RecOut {
    EdgeRec *erec;  // edge table, or
    NegRec *nrec;   // negative table
    const int32_t *src, *dst;
    const uint8_t *heat;  // per node; NULL: every node 255 (never hot)
};

// Without a heat array (imported alias tables carry no degrees) every row is taken as hot:
// the coherent atomic update is correct for any row, only slower.
__device__ __forceinline__ uint32_t heat_of(const RecOut &o, long long v) { return o.heat ? o.heat[v] : 0u; }

__device__ __forceinline__ void write_rec(const RecOut &o, long long i, unsigned long long thr,
                                          int32_t al)
{
    if (o.erec) {
        EdgeRec r;
        r.thr = thr;
        r.alias = al;
        r.src_c = o.src[i];
        r.dst_c = o.dst[i];
        r.src_a = o.src[al];
        r.dst_a = o.dst[al];
        r.heat = heat_of(o, r.src_c) | (heat_of(o, r.dst_c) << 8) | (heat_of(o, r.src_a) << 16) |
                 (heat_of(o, r.dst_a) << 24);
        o.erec[i] = r;
    } else {
        NegRec r;
        r.thr = thr;
        r.alias = al;
        r.heat = heat_of(o, i) | (heat_of(o, al) << 8);
        o.nrec[i] = r;
    }
}

__global__ void k_lights(const double *q, const double *dx, const int32_t *idx, long long nL,
                         long long nH, RecOut o)
{
    long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nL) return;
    long long i = idx[a];
    if (nH == 0) {
        write_rec(o, i, ~0ull, (int32_t)i);
        return;
    }
    const double *D = dx, *X = dx + nL;
    double S = a == 0 ? 0.0 : D[a - 1];
    long long k = count_le(X, nH, S);
    if (k > nH - 1) k = nH - 1;
    write_rec(o, i, prob_to_thr(q[i]), idx[nL + k]);
}

__global__ void k_heavies(const double *dx, const int32_t *idx, long long nL, long long nH, RecOut o)
{
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nH) return;
    const double *D = dx, *X = dx + nL;
    long long i = idx[nL + k];
    if (k == nH - 1) {
        write_rec(o, i, ~0ull, (int32_t)i);
        return;
    }
    long long j = count_start_lt(D, nL, X[k]) - 1;
    double ov = 0.0;
    if (j >= 0) {
        ov = __dsub_rn(D[j], X[k]);
        if (ov < 0.0) ov = 0.0;
    }
    if (ov > 0.0) {
        double p = __dsub_rn(1.0, ov);
        write_rec(o, i, prob_to_thr(p < 0.0 ? 0.0 : p), idx[nL + k + 1]);
    } else {
        write_rec(o, i, ~0ull, (int32_t)i);
    }
}

// ---------------------------------------------------------------------------
// Host driver: one table.
// ---------------------------------------------------------------------------
static lh_status build_one(lh_handle *h, int which, const ScratchLayout &L, char *sc)
{
    hipStream_t s = h->stream;
    long long N = which == LH_ALIAS_EDGE ? h->m : h->n;
    double *wq = (double *)(sc + L.wq);
    double *dx = (double *)(sc + L.dx);
    int32_t *idx = (int32_t *)(sc + L.idx);
    int32_t *lpos = (int32_t *)(sc + L.lpos);
    int32_t *deg = (int32_t *)(sc + L.deg);
    const uint8_t *heat = (const uint8_t *)(h->ws + h->lay.nheat);
    double *lev = (double *)(sc + L.lev);
    int32_t *ilev = (int32_t *)(sc + L.ilev);
    dim3 blk(256), grd((unsigned)LH_CDIV(N, 256));

    // (out-degrees and heats were computed by build_alias before either table)
    if (which == LH_ALIAS_EDGE)
        hipLaunchKernelGGL(k_edge_weights, grd, blk, 0, s, h->w, N, wq);
    else
        hipLaunchKernelGGL(k_neg_weights, grd, blk, 0, s, deg, N, wq);
    chunk_scan<OpNeumaier>(wq, dx, N, lev, s);
    hipLaunchKernelGGL(k_normalise, grd, blk, 0, s, wq, dx, N, lpos, h->status);
    chunk_scan<OpAdd<int32_t>>(lpos, lpos, N, ilev, s);

    int32_t nL32 = 0;
    unsigned int st = 0;
    hipError_t e = hipMemcpyAsync(&nL32, lpos + (N - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&st, h->status, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "alias build");
    if (st & ST_ZERO_TOTAL)
        return fail(h, LH_ERR_ZERO_WEIGHT,
                    which == LH_ALIAS_EDGE ? "total arc weight is zero" : "every node has out-degree 0");
    long long nL = nL32, nH = N - nL;

    hipLaunchKernelGGL(k_split, grd, blk, 0, s, wq, lpos, N, nL, dx, idx);
    if (nL > 0) {
        chunk_scan<OpNeumaier>(dx, dx, nL, lev, s);
        chunk_scan<OpMax>(dx, dx, nL, lev, s);
    }
    if (nH > 0) {
        chunk_scan<OpNeumaier>(dx + nL, dx + nL, nH, lev, s);
        chunk_scan<OpMax>(dx + nL, dx + nL, nH, lev, s);
    }
    RecOut o{which == LH_ALIAS_EDGE ? h->erec : nullptr, which == LH_ALIAS_EDGE ? nullptr : h->nrec,
             h->src, h->dst, heat};
    if (nL > 0)
        hipLaunchKernelGGL(k_lights, dim3((unsigned)LH_CDIV(nL, 256)), blk, 0, s, wq, dx, idx, nL, nH, o);
    if (nH > 0)
        hipLaunchKernelGGL(k_heavies, dim3((unsigned)LH_CDIV(nH, 256)), blk, 0, s, dx, idx, nL, nH, o);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "alias kernels");
    return LH_OK;
}

lh_status build_alias(lh_handle *h, void *scratch, size_t bytes)
{
    ScratchLayout L = scratch_layout(h->n, h->m);
    if (!scratch) return fail(h, LH_ERR_INVALID_ARG, "scratch is NULL");
    if (bytes < L.total) return fail(h, LH_ERR_WORKSPACE_TOO_SMALL, "alias scratch too small");
    h->edge_ready = h->neg_ready = false;
    h->walk.loaded = -1;  // walk roots come from the edge table: pairs made before are stale
    // Out- and in-degrees, the negative weights' canonical scan (for W_nu), and the
    // heat of every node, before either table's records are written.
    {
        char *sc = (char *)scratch;
        hipStream_t s = h->stream;
        int32_t *deg = (int32_t *)(sc + L.deg), *indeg = (int32_t *)(sc + L.indeg);
        double *wq = (double *)(sc + L.wq), *dx = (double *)(sc + L.dx), *lev = (double *)(sc + L.lev);
        dim3 blk(256), gn((unsigned)LH_CDIV(h->n, 256));
        hipLaunchKernelGGL(k_zero_i32, gn, blk, 0, s, deg, h->n);
        hipLaunchKernelGGL(k_zero_i32, gn, blk, 0, s, indeg, h->n);
        hipLaunchKernelGGL(k_degrees, dim3((unsigned)LH_CDIV(h->m, 256)), blk, 0, s, h->src, h->dst, h->m, deg,
                           indeg);
        hipLaunchKernelGGL(k_neg_weights, gn, blk, 0, s, deg, h->n, wq);
        chunk_scan<OpNeumaier>(wq, dx, h->n, lev, s);
        unsigned long long *cnt = (unsigned long long *)(sc + L.cnt);
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(320), 0, s, cnt, 257);
        hipLaunchKernelGGL(k_heat, gn, blk, 0, s, deg, indeg, wq, dx, h->n, h->m, h->p.K,
                           (uint8_t *)(h->ws + h->lay.nheat), cnt);
        unsigned long long host[257];
        hipError_t e = hipMemcpyAsync(host, cnt, sizeof(host), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "degree pass");
        h->n_active = (long long)host[0];
        for (int v = 0; v < 256; ++v) h->heat_count[v] = host[1 + v];
    }
    lh_status st = build_one(h, LH_ALIAS_NEG, L, (char *)scratch);
    if (st != LH_OK) return st;
    h->neg_ready = true;
    st = build_one(h, LH_ALIAS_EDGE, L, (char *)scratch);
    if (st != LH_OK) return st;
    h->edge_ready = true;
    // The scratch may be released by the caller once this work has run.
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "alias build");
    if (!h->cfg_pinned) h->cfg = auto_cfg(h);
    return LH_OK;
}

// ---------------------------------------------------------------------------
// Import / export of (thr, alias) arrays.  Imported alias entries outside [0, N)
// are replaced by the column itself and flagged, so no later kernel reads out of
// bounds.
// ---------------------------------------------------------------------------
__global__ void k_import(const unsigned long long *thr, const int32_t *alias, long long N, RecOut o,
                         unsigned int *status)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int32_t al = alias[i];
    if (al < 0 || (long long)al >= N) {
        atomicOr(status, ST_OUT_OF_RANGE);
        al = (int32_t)i;
    }
    write_rec(o, i, thr[i], al);
}

__global__ void k_export(const EdgeRec *erec, const NegRec *nrec, long long N, unsigned long long *thr,
                         int32_t *alias)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (erec) {
        thr[i] = erec[i].thr;
        alias[i] = erec[i].alias;
    } else {
        thr[i] = nrec[i].thr;
        alias[i] = nrec[i].alias;
    }
}

lh_status import_alias(lh_handle *h, int which, const uint64_t *thr, const int32_t *alias)
{
    if (which == LH_ALIAS_EDGE) h->walk.loaded = -1;  // walk roots come from this table
    long long N = which == LH_ALIAS_EDGE ? h->m : h->n;
    RecOut o{which == LH_ALIAS_EDGE ? h->erec : nullptr, which == LH_ALIAS_EDGE ? nullptr : h->nrec,
             h->src, h->dst, nullptr};
    if (N > 0)
        hipLaunchKernelGGL(k_import, dim3((unsigned)LH_CDIV(N, 256)), dim3(256), 0, h->stream,
                           (const unsigned long long *)thr, alias, N, o, h->status);
    // Imported tables come without degrees: every node is taken as hot (heat 0).
    if (h->n > 0)
        hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)LH_CDIV(h->n, 256)), dim3(256), 0, h->stream,
                           (uint8_t *)(h->ws + h->lay.nheat), h->n, (uint8_t)0);
    for (int v = 0; v < 256; ++v) h->heat_count[v] = 0;
    h->heat_count[0] = (unsigned long long)h->n;
    if (!h->cfg_pinned) h->cfg = auto_cfg(h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "alias import");
    if (which == LH_ALIAS_EDGE)
        h->edge_ready = true;
    else
        h->neg_ready = true;
    return LH_OK;
}

lh_status export_alias(lh_handle *h, int which, uint64_t *thr, int32_t *alias)
{
    long long N = which == LH_ALIAS_EDGE ? h->m : h->n;
    if (N > 0)
        hipLaunchKernelGGL(k_export, dim3((unsigned)LH_CDIV(N, 256)), dim3(256), 0, h->stream,
                           which == LH_ALIAS_EDGE ? h->erec : nullptr,
                           which == LH_ALIAS_EDGE ? nullptr : h->nrec, N,
                           (unsigned long long *)thr, alias);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "alias export");
    return LH_OK;
}

}  // namespace lh

// The alias build of lh_build_alias with its scratch in the static per-device array
// instead of a caller's workspace: the same kernels, handed the array's device address.
// The kernels clear what they accumulate into (degrees, histogram) themselves, and every
// other scratch word is written before it is read, so the contents a previous call left
// do not matter.  Two such calls that overlap on one GPU (two host threads, two streams)
// race on the array.
extern "C" lh_status lh_build_alias_noalloc(lh_handle *h)
{
    if (!h) return LH_ERR_INVALID_ARG;
    if (!h->graph_set) return lh::fail(h, LH_ERR_NOT_BUILT, "lh_set_graph first");
    if (h->m < 1) return lh::fail(h, LH_ERR_ZERO_WEIGHT, "the graph has no arcs");
    // The documented limits; scratch_layout(2^21, 2^21) is 64.03 MiB, within the array.
    const lh::ScratchLayout L = lh::scratch_layout(h->n, h->m);
    if (h->n > lh::kNoAllocMaxItems || h->m > lh::kNoAllocMaxItems || L.total > lh::kNoAllocScratchBytes)
        return lh::fail(h, LH_ERR_INVALID_ARG,
                        "graph too large for the static build scratch (65 MiB: n and m up to 2^21 each)");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != h->device) (void)hipSetDevice(h->device);
    lh_status st = LH_OK;
    hipError_t e = lh::noalloc_scratch_setup(h->device);
    void *ptr = lh::noalloc_scratch(h->device);
    if (e != hipSuccess || !ptr)
        st = lh::hip_fail(h, e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch address");
    else
        st = lh::build_alias(h, ptr, lh::kNoAllocScratchBytes);
    if (prev >= 0 && prev != h->device) (void)hipSetDevice(prev);
    return st;
}
