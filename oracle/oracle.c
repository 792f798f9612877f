/*
 * CPU oracle for LINE-style edge-sampled SGD.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header, table or
 * constant generator with the GPU library, and it includes nothing from it.
 *
 * Paper: "NOMAD: Generating Embeddings for Massive Distributed Graphs" (arXiv 2604.09419).
 *   - Eq. (1), Sec. IV-A (Distributed Training): negatives follow q(v) ~ d(v)^0.75 with
 *     d(v) the out-degree.
 *   - Algorithm 1 (local updates) and Eqs. (2)-(3): per positive pair
 *     g = eta (1 - sigma(U[u].C[v])); per negative g = -eta alpha_neg sigma(U[u].C[v-]);
 *     LineUpdate adds g*C - eta*lambda*U to U[u] and g*U0 - eta*lambda*C to the context
 *     row, where U0 is the vertex row before the update.
 *   - Eq. (4): a row's batch update is the sum of the per-pair contributions computed
 *     against the copy fetched at the start of the batch (the SNAPSHOT mode below).
 *   - Algorithm 3 (GeneratePairs), root selection: a positive pair is an edge drawn from
 *     the weight-normalised edge distribution.
 *   - Algorithms 2-3 (RandomWalk, GeneratePairs), Sec. IV-B: positive pairs from random
 *     walks rooted at such an edge (the walk pair source below).
 *   - Sec. IV-C (variants of random walks), Augmented-Pair: a pool of walk pairs
 *     collected before training and expanded by recombination (the pair pool below).
 *   - Sec. V-A (NOMAD hyperparameters): single-precision SGD, eta = 0.025.
 *
 * Floating point: everything here is IEEE binary64 except the Hogwild timing mode,
 * which is binary32.  Build with -ffp-contract=off and without -ffast-math.
 *
 * Readings of the paper that this file commits to (the paper leaves them open):
 *   - sigma(U[u], C[v]) is the logistic function of the dot product.
 *   - All 1+K dot products of one sample use the vertex row as it was before the
 *     sample; the row receives the sum of the 1+K LineUpdate increments.
 *   - lambda (weight decay) applies once per pair, i.e. 1+K times to U[u] per sample.
 *   - First-order proximity uses one table U1 at both ends of every pair.
 *   - The alias encoding, the counter-based generator (Philox4x64-10), the canonical
 *     chunked scan and the linear learning-rate decay are this library's own choices;
 *     the paper names no method for its discrete distributions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as     */
/* easy as 1, 2, 3", SC'11).  Ten rounds of the 4x64 S-box; the key is bumped  */
/* by the two Weyl constants between rounds.                                   */
/* ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void or_philox4x64_10(uint64_t key0, uint64_t key1, const uint64_t ctr[4], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key0, k1 = key1;
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        u128 p0 = (u128)PHILOX_M0 * c0;
        u128 p1 = (u128)PHILOX_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------- */
/* Canonical chunked scan.                                                     */
/*                                                                             */
/* cscan(x[0..N)): chunk c covers [c*1024, min((c+1)*1024, N)).  Inside a chunk */
/* a left-to-right Neumaier-compensated running sum gives loc[i] = s + comp.   */
/* tot[c] is the chunk's last loc.  The offsets are the exclusive form of      */
/* cscan(tot), applied recursively, and out[i] = loc[i] for chunk 0 and        */
/* fl(off[c] + loc[i]) otherwise.  The association order is fixed, so any      */
/* implementation that follows it reproduces every bit.                        */
/* ------------------------------------------------------------------------- */
#define OR_CHUNK 1024

void or_cscan(const double *x, int64_t n, double *out)
{
    if (n <= 0) return;
    int64_t nchunks = (n + OR_CHUNK - 1) / OR_CHUNK;
    double *tot = (double *)malloc(sizeof(double) * (size_t)nchunks);
    for (int64_t c = 0; c < nchunks; c++) {
        int64_t lo = c * OR_CHUNK, hi = lo + OR_CHUNK < n ? lo + OR_CHUNK : n;
        double s = 0.0, comp = 0.0;
        for (int64_t i = lo; i < hi; i++) {
            double xi = x[i];
            double t = s + xi;
            if (fabs(s) >= fabs(xi))
                comp += (s - t) + xi;
            else
                comp += (xi - t) + s;
            s = t;
            out[i] = s + comp;
        }
        tot[c] = out[hi - 1];
    }
    if (nchunks > 1) {
        double *inc = (double *)malloc(sizeof(double) * (size_t)nchunks);
        or_cscan(tot, nchunks, inc);
        for (int64_t c = 1; c < nchunks; c++) {
            double off = inc[c - 1];
            int64_t lo = c * OR_CHUNK, hi = lo + OR_CHUNK < n ? lo + OR_CHUNK : n;
            for (int64_t i = lo; i < hi; i++) out[i] = off + out[i];
        }
        free(inc);
    }
    free(tot);
}

/* Monotone form: the running maximum of the canonical scan.  Max is exact, so
 * the result does not depend on evaluation order either. */
void or_mscan(const double *x, int64_t n, double *out)
{
    or_cscan(x, n, out);
    for (int64_t i = 1; i < n; i++)
        if (out[i] < out[i - 1]) out[i] = out[i - 1];
}

/* ------------------------------------------------------------------------- */
/* Negative-sampling weights, Eq. (1): nu_v = d(v)^0.75 with d the out-degree. */
/* d^0.75 = sqrt(d) * sqrt(sqrt(d)); every operation is correctly rounded.     */
/* ------------------------------------------------------------------------- */
void or_out_degree(const int32_t *src, int64_t m, int64_t n, int64_t *deg)
{
    for (int64_t v = 0; v < n; v++) deg[v] = 0;
    for (int64_t a = 0; a < m; a++) deg[src[a]] += 1;
}

void or_neg_weights(const int64_t *deg, int64_t n, double *nu)
{
    for (int64_t v = 0; v < n; v++) {
        double s = sqrt((double)deg[v]);
        double t = sqrt(s);
        nu[v] = s * t;
    }
}

/* ------------------------------------------------------------------------- */
/* Alias table over N items with weights w (Walker 1977 / Vose 1991), built in */
/* the closed form of the sweeping construction (Huebschle-Schneider and       */
/* Sanders, "Parallel Weighted Random Sampling"):                              */
/*   W = last element of cscan(w); q_i = fl(fl(w_i * N) / W)                    */
/*   lights L = {q_i < 1}, heavies H = {q_i >= 1}, each in index order          */
/*   D = mscan(1 - q over L), X = mscan(q - 1 over H), S_a = (a ? D[a-1] : 0)    */
/*   light a:  prob = q, alias = H[min(#{k : X[k] <= S_a}, |H|-1)]              */
/*   heavy k < |H|-1: j = #{a : S_a < X[k]} - 1, o = j >= 0 ? max(0, D[j]-X[k]) */
/*             : 0; o > 0 gives prob = max(0, 1-o), alias = H[k+1], else prob 1 */
/*   last heavy (or every item when H is empty): prob = 1, alias = self         */
/*   thr = prob >= 1 ? 2^64-1 : (uint64)(prob * 2^64)                           */
/* Returns 0, or 1 when the total weight is not a positive finite number.      */
/* ------------------------------------------------------------------------- */
static int64_t count_le(const double *X, int64_t nH, double s) /* #{k : X[k] <= s} */
{
    int64_t lo = 0, hi = nH;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (X[mid] <= s) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int64_t count_start_lt(const double *D, int64_t nL, double x) /* #{a : S_a < x} */
{
    if (nL == 0 || !(0.0 < x)) return 0;
    int64_t lo = 0, hi = nL - 1; /* S_a = D[a-1] for a in [1, nL) */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (D[mid] < x) lo = mid + 1; else hi = mid;
    }
    return 1 + lo;
}

int or_alias_build(const double *w, int64_t N, uint64_t *thr, int32_t *alias)
{
    if (N <= 0) return 1;
    double *scan = (double *)malloc(sizeof(double) * (size_t)N);
    or_cscan(w, N, scan);
    double W = scan[N - 1];
    free(scan);
    if (!(W > 0.0) || !isfinite(W)) return 1;

    double *q = (double *)malloc(sizeof(double) * (size_t)N);
    int64_t nL = 0, nH = 0;
    for (int64_t i = 0; i < N; i++) {
        q[i] = (w[i] * (double)N) / W;
        if (q[i] < 1.0) nL++; else nH++;
    }
    int64_t *L = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nL ? nL : 1));
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nH ? nH : 1));
    double *dl = (double *)malloc(sizeof(double) * (size_t)(nL ? nL : 1));
    double *eh = (double *)malloc(sizeof(double) * (size_t)(nH ? nH : 1));
    nL = nH = 0;
    for (int64_t i = 0; i < N; i++) {
        if (q[i] < 1.0) { L[nL] = i; dl[nL] = 1.0 - q[i]; nL++; }
        else            { H[nH] = i; eh[nH] = q[i] - 1.0; nH++; }
    }
    double *D = (double *)malloc(sizeof(double) * (size_t)(nL ? nL : 1));
    double *X = (double *)malloc(sizeof(double) * (size_t)(nH ? nH : 1));
    or_mscan(dl, nL, D);
    or_mscan(eh, nH, X);

    double *prob = (double *)malloc(sizeof(double) * (size_t)N);
    if (nH == 0) {
        for (int64_t i = 0; i < N; i++) { prob[i] = 1.0; alias[i] = (int32_t)i; }
    } else {
        for (int64_t a = 0; a < nL; a++) {
            double S = a == 0 ? 0.0 : D[a - 1];
            int64_t k = count_le(X, nH, S);
            if (k > nH - 1) k = nH - 1;
            prob[L[a]] = q[L[a]];
            alias[L[a]] = (int32_t)H[k];
        }
        for (int64_t k = 0; k < nH; k++) {
            int64_t i = H[k];
            if (k == nH - 1) { prob[i] = 1.0; alias[i] = (int32_t)i; continue; }
            int64_t j = count_start_lt(D, nL, X[k]) - 1;
            double o = 0.0;
            if (j >= 0) { o = D[j] - X[k]; if (o < 0.0) o = 0.0; }
            if (o > 0.0) {
                double p = 1.0 - o;
                prob[i] = p < 0.0 ? 0.0 : p;
                alias[i] = (int32_t)H[k + 1];
            } else {
                prob[i] = 1.0;
                alias[i] = (int32_t)i;
            }
        }
    }
    for (int64_t i = 0; i < N; i++)
        thr[i] = prob[i] >= 1.0 ? UINT64_MAX : (uint64_t)(prob[i] * 18446744073709551616.0);

    free(prob); free(D); free(X); free(dl); free(eh); free(L); free(H); free(q);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Drawing.  Sample s, slot j (0 = the positive edge, 1..K = negatives) takes  */
/* Block(key = (seed, graph_id), ctr = (s, j, 0, 0)).  col = floor(x0 * N /    */
/* 2^64); the item is col when x1 < thr[col], else alias[col].  Slot 0's item  */
/* is an arc a, giving (u, v) = (src[a], dst[a]) (Algorithm 3, root edge);    */
/* slots 1..K are negatives drawn i.i.d. from Eq. (1) (Algorithm 1).           */
/* ------------------------------------------------------------------------- */
static inline int64_t draw(const uint64_t *thr, const int32_t *alias, int64_t N,
                           uint64_t x0, uint64_t x1)
{
    int64_t col = (int64_t)(((u128)x0 * (uint64_t)N) >> 64);
    return x1 < thr[col] ? col : (int64_t)alias[col];
}

/* Exposed for the tests: the draw of one item from crafted words. */
int64_t or_draw_item(const uint64_t *thr, const int32_t *alias, int64_t N, uint64_t x0, uint64_t x1)
{
    return draw(thr, alias, N, x0, x1);
}

typedef struct {
    int64_t n, m;
    const int32_t *src, *dst;
    const uint64_t *ethr; const int32_t *ealias;
    const uint64_t *nthr; const int32_t *nalias;
    uint64_t seed; uint32_t graph_id;
    int K;
    /* Positive pairs from random walks instead of arc draws: the pair of sample s is     */
    /* (pu[s - pfirst], pv[s - pfirst]); NULL: slot 0 draws an arc.                       */
    const int32_t *pu, *pv;
    uint64_t pfirst;
} or_graph;

static void draw_tuple(const or_graph *g, uint64_t s, int32_t *u, int32_t *v, int32_t *neg)
{
    uint64_t ctr[4] = {s, 0, 0, 0}, x[4];
    if (g->pu) {
        *u = g->pu[s - g->pfirst];
        *v = g->pv[s - g->pfirst];
    } else {
        or_philox4x64_10(g->seed, (uint64_t)g->graph_id, ctr, x);
        int64_t a = draw(g->ethr, g->ealias, g->m, x[0], x[1]);
        *u = g->src[a];
        *v = g->dst[a];
    }
    for (int j = 1; j <= g->K; j++) {
        ctr[1] = (uint64_t)j;
        or_philox4x64_10(g->seed, (uint64_t)g->graph_id, ctr, x);
        neg[j - 1] = (int32_t)draw(g->nthr, g->nalias, g->n, x[0], x[1]);
    }
}

void or_sample(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
               const uint64_t *ethr, const int32_t *ealias,
               const uint64_t *nthr, const int32_t *nalias,
               uint64_t seed, uint32_t graph_id, int K,
               uint64_t first, uint64_t count, int32_t *u, int32_t *v, int32_t *neg)
{
    or_graph g = {n, m, src, dst, ethr, ealias, nthr, nalias, seed, graph_id, K, NULL, NULL, 0};
    for (uint64_t i = 0; i < count; i++)
        draw_tuple(&g, first + i, &u[i], &v[i], &neg[i * (uint64_t)K]);
}

/* The negatives alone (a negative table needs no arcs): slot j = 1..K of sample s
 * from the same blocks as draw_tuple. */
void or_sample_negatives(int64_t n, const uint64_t *nthr, const int32_t *nalias,
                         uint64_t seed, uint32_t graph_id, int K,
                         uint64_t first, uint64_t count, int32_t *neg)
{
    for (uint64_t i = 0; i < count; i++) {
        for (int j = 1; j <= K; j++) {
            uint64_t ctr[4] = {first + i, (uint64_t)j, 0, 0}, x[4];
            or_philox4x64_10(seed, (uint64_t)graph_id, ctr, x);
            neg[i * (uint64_t)K + (uint64_t)(j - 1)] = (int32_t)draw(nthr, nalias, n, x[0], x[1]);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Initial embeddings: uniform on [-0.5/d, 0.5/d).  Element (t, r, c) of table  */
/* t (0 = U, 1 = C, 2 = U1) is word c mod 4 of Block(key = (seed, 2^32 | g),    */
/* ctr = (r, c / 4, t, 0)); val = ((x >> 40) - 2^23) * 2^-24 / d, rounded once   */
/* to binary32 (exact when d is a power of two).                               */
/* ------------------------------------------------------------------------- */
void or_init_table(float *out, int t, int64_t rows, int d, uint64_t seed, uint32_t graph_id)
{
    for (int64_t r = 0; r < rows; r++) {
        for (int c4 = 0; c4 < (d + 3) / 4; c4++) {
            uint64_t ctr[4] = {(uint64_t)r, (uint64_t)c4, (uint64_t)t, 0}, x[4];
            or_philox4x64_10(seed, (1ULL << 32) | graph_id, ctr, x);
            for (int k = 0; k < 4 && c4 * 4 + k < d; k++) {
                double val = ((double)((int64_t)(x[k] >> 40) - 8388608) * 0x1p-24) / (double)d;
                out[r * d + c4 * 4 + k] = (float)val;
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Training in binary64.                                                       */
/*   eta_s = eta0 * (1 - s / T)                                                 */
/*   order 2: (A, B) = (U, C); order 1: A = B = U1                              */
/*   with a = A[u], b_0 = B[v], b_k = B[n_k] taken before the sample:           */
/*     x_j = a . b_j, g_0 = eta_s (1 - sigma(x_0)), g_k = -eta_s alpha sigma(x_k) */
/*     A[u]   += sum_j (g_j b_j - eta_s lambda a)                                */
/*     B[v]   += g_0 a - eta_s lambda b_0                                        */
/*     B[n_k] += g_k a - eta_s lambda b_k                                        */
/* mode 0 (SEQ) applies each sample's increments at once.  mode 1 (SNAPSHOT)   */
/* groups samples into batches [bB, (b+1)B) and computes every increment of a  */
/* batch from the tables as they were at its start, summing per row (Eq. (4)) */
/* in (sample, slot) order before adding the sum to the row.                   */
/* ------------------------------------------------------------------------- */
static inline double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

typedef struct {
    int d, K, orders;
    double eta0, lambda, alpha;
    uint64_t T;
} or_hyper;

/* Increments of one sample and one order into dA (d) and dB ((1+K) x d). */
static void sample_increments(const or_hyper *h, double eta, const double *A, const double *B,
                              int32_t u, const int32_t *ids, double *dA, double *dB)
{
    int d = h->d, K = h->K;
    const double *a = A + (int64_t)u * d;
    for (int c = 0; c < d; c++) dA[c] = 0.0;
    for (int j = 0; j <= K; j++) {
        const double *b = B + (int64_t)ids[j] * d;
        double x = 0.0;
        for (int c = 0; c < d; c++) x += a[c] * b[c];
        double g = j == 0 ? eta * (1.0 - sigmoid(x)) : -eta * h->alpha * sigmoid(x);
        for (int c = 0; c < d; c++) {
            dA[c] += g * b[c] - eta * h->lambda * a[c];
            dB[j * d + c] = g * a[c] - eta * h->lambda * b[c];
        }
    }
}

/* Exposed for the tests: apply one given tuple (u; v = ids[0]; n_k = ids[k]) to the
 * tables A and B in the SEQ manner, with step size eta. */
void or_apply_tuple(double *A, double *B, int d, int K, int32_t u, const int32_t *ids,
                    double eta, double lambda, double alpha)
{
    or_hyper h = {d, K, 2, 0.0, lambda, alpha, 1};
    double *dA = (double *)malloc(sizeof(double) * (size_t)d);
    double *dB = (double *)malloc(sizeof(double) * (size_t)d * (size_t)(K + 1));
    sample_increments(&h, eta, A, B, u, ids, dA, dB);
    for (int c = 0; c < d; c++) A[(int64_t)u * d + c] += dA[c];
    for (int j = 0; j <= K; j++)
        for (int c = 0; c < d; c++) B[(int64_t)ids[j] * d + c] += dB[j * d + c];
    free(dA); free(dB);
}

static int train_range(const or_graph *gp, const or_hyper *hp, double *U, double *C, double *U1,
                       uint64_t first, uint64_t count, int mode, uint64_t batch)
{
    const or_graph g = *gp;
    const or_hyper h = *hp;
    const int64_t n = g.n;
    const int d = h.d, K = h.K, orders = h.orders;
    const double eta0 = h.eta0;
    const uint64_t T = h.T;
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K + 1));
    double *dA = (double *)malloc(sizeof(double) * (size_t)d);
    double *dB = (double *)malloc(sizeof(double) * (size_t)d * (size_t)(K + 1));

    if (mode == 0) {
        for (uint64_t s = first; s < first + count; s++) {
            int32_t u;
            draw_tuple(&g, s, &u, &ids[0], &ids[1]);
            double eta = eta0 * (1.0 - (double)s / (double)T);
            for (int o = 2; o >= 1; o--) {
                if (!(orders & o)) continue;
                double *A = o == 2 ? U : U1, *B = o == 2 ? C : U1;
                sample_increments(&h, eta, A, B, u, ids, dA, dB);
                for (int c = 0; c < d; c++) A[(int64_t)u * d + c] += dA[c];
                for (int j = 0; j <= K; j++)
                    for (int c = 0; c < d; c++) B[(int64_t)ids[j] * d + c] += dB[j * d + c];
            }
        }
    } else {
        /* Per-row sums for the three tables, and the list of rows touched. */
        double *acc[3] = {0, 0, 0};
        char *touched[3] = {0, 0, 0};
        int64_t *list[3] = {0, 0, 0}, nlist[3] = {0, 0, 0};
        double *tab[3] = {U, C, U1};
        for (int t = 0; t < 3; t++) {
            if (!tab[t]) continue;
            acc[t] = (double *)calloc((size_t)n * (size_t)d, sizeof(double));
            touched[t] = (char *)calloc((size_t)n, 1);
            list[t] = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        }
        uint64_t end = first + count;
        uint64_t s = first;
        while (s < end) {
            uint64_t bend = (s / batch + 1) * batch;
            if (bend > end) bend = end;
            for (; s < bend; s++) {
                int32_t u;
                draw_tuple(&g, s, &u, &ids[0], &ids[1]);
                double eta = eta0 * (1.0 - (double)s / (double)T);
                for (int o = 2; o >= 1; o--) {
                    if (!(orders & o)) continue;
                    int ta = o == 2 ? 0 : 2, tb = o == 2 ? 1 : 2;
                    sample_increments(&h, eta, tab[ta], tab[tb], u, ids, dA, dB);
                    if (!touched[ta][u]) { touched[ta][u] = 1; list[ta][nlist[ta]++] = u; }
                    for (int c = 0; c < d; c++) acc[ta][(int64_t)u * d + c] += dA[c];
                    for (int j = 0; j <= K; j++) {
                        int32_t r = ids[j];
                        if (!touched[tb][r]) { touched[tb][r] = 1; list[tb][nlist[tb]++] = r; }
                        for (int c = 0; c < d; c++) acc[tb][(int64_t)r * d + c] += dB[j * d + c];
                    }
                }
            }
            for (int t = 0; t < 3; t++) {
                if (!tab[t]) continue;
                for (int64_t i = 0; i < nlist[t]; i++) {
                    int64_t r = list[t][i];
                    for (int c = 0; c < d; c++) {
                        tab[t][r * d + c] += acc[t][r * d + c];
                        acc[t][r * d + c] = 0.0;
                    }
                    touched[t][r] = 0;
                }
                nlist[t] = 0;
            }
        }
        for (int t = 0; t < 3; t++) { free(acc[t]); free(touched[t]); free(list[t]); }
    }
    free(ids); free(dA); free(dB);
    return 0;
}

int or_train(const int32_t *src, const int32_t *dst, int64_t n, int64_t m,
             const uint64_t *ethr, const int32_t *ealias,
             const uint64_t *nthr, const int32_t *nalias,
             uint64_t seed, uint32_t graph_id,
             int d, int K, int orders, double eta0, double lambda, double alpha, uint64_t T,
             double *U, double *C, double *U1,
             uint64_t first, uint64_t count, int mode, uint64_t batch)
{
    if (d <= 0 || K < 0 || T == 0 || (orders & 3) == 0) return 1;
    if ((orders & 2) && (!U || !C)) return 1;
    if ((orders & 1) && !U1) return 1;
    if (mode == 1 && batch == 0) return 1;
    or_graph g = {n, m, src, dst, ethr, ealias, nthr, nalias, seed, graph_id, K, NULL, NULL, 0};
    or_hyper h = {d, K, orders, eta0, lambda, alpha, T};
    return train_range(&g, &h, U, C, U1, first, count, mode, batch);
}

/* ------------------------------------------------------------------------- */
/* Random-walk positive pairs (Sec. IV-B: Algorithm 2, RandomWalk, and          */
/* Algorithm 3, GeneratePairs) on one process, where every vertex is local, so  */
/* the walk never stops at a remote vertex (the "Local" variant over the whole  */
/* graph).                                                                     */
/*                                                                             */
/* Walk graph: the undirected graph of the arcs, as the paper walks undirected */
/* graphs.  Entry e < m is arc e forwards (tail src[e], head dst[e]); entry     */
/* m + e is arc e backwards (tail dst[e], head src[e]); both weigh w[e].  The   */
/* neighbourhood N(x) lists the entries with tail x in increasing entry index:  */
/* CSR rows off[x] .. off[x+1], heads nbr[], weights wt[].                      */
/*                                                                             */
/* discrete(N(x)) is an alias table over the row's weights (or_alias_build on   */
/* the row, items numbered from 0 within the row).  A row whose weights sum to  */
/* zero gets prob 1 and itself everywhere; no walk reaches it, since every     */
/* step leaves along an entry of positive weight and the reverse entry then    */
/* has that weight too.                                                        */
/*                                                                             */
/* Walk k, vertices w_0 .. w_{L-1} (L = walk length: Algorithm 2 counts the    */
/* visited vertices, root pair included, up to it), Philox4x64-10 with key      */
/* (seed, 5 * 2^32 | graph_id):                                                 */
/*   block (k, 0, 0, 0) draws the root arc a from the edge table (Algorithm 3,  */
/*   the weight-normalised edge distribution): w_0 = src[a], w_1 = dst[a];      */
/*   block (k, t, 0, 0), t = 1 .. L-2, draws w_{t+1} from discrete(N(w_t)).     */
/* Pairs of a walk: (w_i, w_{i+delta}) for delta = 1 .. W-1 (window W; W = 2   */
/* gives the consecutive pairs Algorithm 2 collects into its path), numbered    */
/* p = sum_{delta' < delta} (L - delta') + i; P pairs per walk.                 */
/* Sample order (Algorithm 3 shuffles the pairs of a batch): walks come in      */
/* batches of Bw, and sample s = b Bw P + p Bw + j is pair p of walk b Bw + j,  */
/* so consecutive samples come from different walks.                            */
/* ------------------------------------------------------------------------- */
#define OR_WALK_TAG 5ULL

int or_walk_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                int64_t *off, int32_t *nbr, double *wt)
{
    if (n < 1 || m < 0) return 1;
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t x = 0; x <= n; x++) off[x] = 0;
    for (int64_t e = 0; e < m; e++) { off[src[e] + 1]++; off[dst[e] + 1]++; }
    for (int64_t x = 0; x < n; x++) off[x + 1] += off[x];
    for (int64_t e = 0; e < 2 * m; e++) {
        int64_t a = e < m ? e : e - m;
        int32_t tail = e < m ? src[a] : dst[a], head = e < m ? dst[a] : src[a];
        int64_t pos = off[tail] + fill[tail]++;
        nbr[pos] = head;
        wt[pos] = (double)w[a];
    }
    free(fill);
    return 0;
}

void or_walk_alias(int64_t n, const int64_t *off, const double *wt, uint64_t *thr, int32_t *alias)
{
    for (int64_t x = 0; x < n; x++) {
        int64_t lo = off[x], len = off[x + 1] - off[x];
        if (len == 0) continue;
        if (or_alias_build(wt + lo, len, thr + lo, alias + lo) != 0) {
            for (int64_t i = 0; i < len; i++) { thr[lo + i] = UINT64_MAX; alias[lo + i] = (int32_t)i; }
        }
    }
}

typedef struct {
    int64_t n, m;
    const int32_t *src, *dst;
    const uint64_t *ethr; const int32_t *ealias;
    const int64_t *off; const int32_t *nbr;
    const uint64_t *wthr; const int32_t *walias;
    uint64_t seed; uint32_t graph_id;
    int L, W;
    int64_t Bw;
} or_walker;

static void walk_vertices(const or_walker *wk, uint64_t k, int32_t *vert)
{
    uint64_t key1 = (OR_WALK_TAG << 32) | (uint64_t)wk->graph_id, ctr[4] = {k, 0, 0, 0}, x[4];
    or_philox4x64_10(wk->seed, key1, ctr, x);
    int64_t a = draw(wk->ethr, wk->ealias, wk->m, x[0], x[1]);
    vert[0] = wk->src[a];
    vert[1] = wk->dst[a];
    for (int t = 1; t + 1 < wk->L; t++) {
        ctr[1] = (uint64_t)t;
        or_philox4x64_10(wk->seed, key1, ctr, x);
        int64_t lo = wk->off[vert[t]], len = wk->off[vert[t] + 1] - lo;
        int64_t item = draw(wk->wthr + lo, wk->walias + lo, len, x[0], x[1]);
        vert[t + 1] = wk->nbr[lo + item];
    }
}

static int64_t walk_pairs_per_walk(int L, int W)
{
    int64_t P = 0;
    for (int delta = 1; delta < W; delta++) P += L - delta;
    return P;
}

/* The pair (first, second position) with number p of a walk. */
static void walk_pair_positions(int L, int W, int64_t p, int *i, int *j)
{
    int delta = 1;
    while (delta < W && p >= L - delta) { p -= L - delta; delta++; }
    *i = (int)p;
    *j = (int)p + delta;
}

static int walker_ok(const or_walker *wk)
{
    return wk->L >= 2 && wk->W >= 2 && wk->W <= wk->L && wk->Bw >= 1 && wk->m >= 1;
}

/* The pairs of walk batch b in sample order: pu/pv[p Bw + j] = pair p of walk b Bw + j. */
static void fill_walk_batch(const or_walker *wk, uint64_t b, int32_t *pu, int32_t *pv)
{
    const int L = wk->L, W = wk->W;
    const uint64_t Bw = (uint64_t)wk->Bw, P = (uint64_t)walk_pairs_per_walk(L, W);
    int32_t *vert = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    for (uint64_t j = 0; j < Bw; j++) {
        walk_vertices(wk, b * Bw + j, vert);
        for (uint64_t p = 0; p < P; p++) {
            int a, c;
            walk_pair_positions(L, W, (int64_t)p, &a, &c);
            pu[p * Bw + j] = vert[a];
            pv[p * Bw + j] = vert[c];
        }
    }
    free(vert);
}

/* The positive pairs of samples [first, first + count). */
int or_walk_pairs(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                  const uint64_t *ethr, const int32_t *ealias,
                  const int64_t *off, const int32_t *nbr, const uint64_t *wthr, const int32_t *walias,
                  uint64_t seed, uint32_t graph_id, int L, int W, int64_t Bw,
                  uint64_t first, uint64_t count, int32_t *u, int32_t *v)
{
    or_walker wk = {n, m, src, dst, ethr, ealias, off, nbr, wthr, walias, seed, graph_id, L, W, Bw};
    if (!walker_ok(&wk)) return 1;
    const uint64_t P = (uint64_t)walk_pairs_per_walk(L, W), per = (uint64_t)Bw * P;
    int32_t *vert = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    uint64_t have = UINT64_MAX;
    for (uint64_t i = 0; i < count; i++) {
        uint64_t s = first + i, b = s / per, r = s % per, p = r / (uint64_t)Bw, j = r % (uint64_t)Bw;
        uint64_t k = b * (uint64_t)Bw + j;
        if (k != have) { walk_vertices(&wk, k, vert); have = k; }
        int a, c;
        walk_pair_positions(L, W, (int64_t)p, &a, &c);
        u[i] = vert[a];
        v[i] = vert[c];
    }
    free(vert);
    return 0;
}

/* Whole walks k0 .. k0 + nwalks - 1: vertex t of walk k into vert[(k - k0) L + t]. */
int or_walk_vertices(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     const uint64_t *ethr, const int32_t *ealias,
                     const int64_t *off, const int32_t *nbr, const uint64_t *wthr, const int32_t *walias,
                     uint64_t seed, uint32_t graph_id, int L, uint64_t k0, uint64_t nwalks, int32_t *vert)
{
    or_walker wk = {n, m, src, dst, ethr, ealias, off, nbr, wthr, walias, seed, graph_id, L, 2, 1};
    if (!walker_ok(&wk)) return 1;
    for (uint64_t k = 0; k < nwalks; k++) walk_vertices(&wk, k0 + k, vert + k * (uint64_t)L);
    return 0;
}

/* Training (or_train) with the positive pairs of the walks: Algorithm 3 generates the
 * pairs of each walk batch, then Algorithm 1 trains them in sample order.  SNAPSHOT needs
 * every batch [bB, (b+1)B) inside one walk batch: Bw P a multiple of B. */
int or_train_walk(const int32_t *src, const int32_t *dst, int64_t n, int64_t m,
                  const uint64_t *ethr, const int32_t *ealias,
                  const uint64_t *nthr, const int32_t *nalias,
                  const int64_t *off, const int32_t *nbr, const uint64_t *wthr, const int32_t *walias,
                  int L, int W, int64_t Bw,
                  uint64_t seed, uint32_t graph_id,
                  int d, int K, int orders, double eta0, double lambda, double alpha, uint64_t T,
                  double *U, double *C, double *U1,
                  uint64_t first, uint64_t count, int mode, uint64_t batch)
{
    if (d <= 0 || K < 0 || T == 0 || (orders & 3) == 0) return 1;
    if ((orders & 2) && (!U || !C)) return 1;
    if ((orders & 1) && !U1) return 1;
    if (mode == 1 && batch == 0) return 1;
    or_walker wk = {n, m, src, dst, ethr, ealias, off, nbr, wthr, walias, seed, graph_id, L, W, Bw};
    if (!walker_ok(&wk)) return 1;
    const uint64_t per = (uint64_t)Bw * (uint64_t)walk_pairs_per_walk(L, W);
    if (mode == 1 && per % batch != 0) return 1;
    or_hyper h = {d, K, orders, eta0, lambda, alpha, T};
    int32_t *pu = (int32_t *)malloc(sizeof(int32_t) * (size_t)per);
    int32_t *pv = (int32_t *)malloc(sizeof(int32_t) * (size_t)per);
    const uint64_t end = first + count;
    int rc = 0;
    for (uint64_t s = first; s < end && rc == 0;) {
        uint64_t b = s / per, b0 = b * per, b1 = b0 + per;
        fill_walk_batch(&wk, b, pu, pv);
        or_graph g = {n, m, src, dst, ethr, ealias, nthr, nalias, seed, graph_id, K, pu, pv, b0};
        uint64_t stop = b1 < end ? b1 : end;
        rc = train_range(&g, &h, U, C, U1, s, stop - s, mode, batch);
        s = stop;
    }
    free(pu); free(pv);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* bfloat16 storage (the precision extension of the embedding tables): every   */
/* value written to a table is the binary64 result rounded to binary32 (to     */
/* nearest) and then stochastically to bfloat16 -- 16 random bits are added to */
/* the binary32 pattern and the low 16 bits dropped, so the magnitude rounds up */
/* with probability equal to its distance from the lower neighbour, in ulps    */
/* (NaN stays a quiet NaN).  The bits come from Philox4x64-10 with key         */
/* (seed, 2^34 | graph_id): the value written by write w of sample s (w = 16 o  */
/* + slot, slot 0 the vertex row, 1 + j context slot j, o the order) to element */
/* c uses 16-bit chunk c mod 16 of block (s, w, c / 16, stream); stream numbers */
/* independent rounding streams of one run (0 by default).                     */
/* ------------------------------------------------------------------------- */
static double sr_bf16(double x, uint16_t r)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        u = (u | 0x00400000u) & 0xffff0000u;
    } else {
        u = (u + (uint32_t)r) & 0xffff0000u;
    }
    memcpy(&f, &u, 4);
    return (double)f;
}

/* Exposed for the tests: the stochastic rounding of x with 16 given bits. */
double or_sr_bf16(double x, uint32_t r) { return sr_bf16(x, (uint16_t)(r & 0xffffu)); }

/* Nearest bfloat16 (ties to even) of the binary32 rounding of each x: the stored
 * initial values. */
void or_bf16_rne(double *x, int64_t n)
{
    for (int64_t i = 0; i < n; i++) {
        float f = (float)x[i];
        uint32_t u;
        memcpy(&u, &f, 4);
        if ((u & 0x7fffffffu) > 0x7f800000u) {
            u = (u | 0x00400000u) & 0xffff0000u;
        } else {
            u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
        }
        memcpy(&f, &u, 4);
        x[i] = (double)f;
    }
}

/* Add inc to row r of X in place, each element written as sr_bf16 with the bits of
 * write w of sample s. */
static void write_row_bf16(double *X, int64_t r, const double *inc, int d, uint64_t seed,
                           uint32_t graph_id, uint64_t s, uint64_t w, uint64_t stream)
{
    uint64_t x[4] = {0, 0, 0, 0};
    for (int c = 0; c < d; c++) {
        if (c % 16 == 0) {
            uint64_t ctr[4] = {s, w, (uint64_t)(c / 16), stream};
            or_philox4x64_10(seed, (4ULL << 32) | graph_id, ctr, x);
        }
        uint16_t bits = (uint16_t)(x[(c % 16) / 4] >> (16 * (c % 4)));
        X[r * d + c] = sr_bf16(X[r * d + c] + inc[c], bits);
    }
}

/* SEQ mode with bfloat16 tables: or_train's mode 0 (the increments of a sample
 * from the rows before it, in binary64), each row of each order written back
 * through write_row_bf16 in the order vertex row, then context slots 0..K. */
static void train_range_bf16(const or_graph *gp, const or_hyper *hp, double *U, double *C, double *U1,
                             uint64_t first, uint64_t count, uint64_t stream)
{
    const or_graph g = *gp;
    const or_hyper h = *hp;
    const int d = h.d, K = h.K, orders = h.orders;
    const double eta0 = h.eta0;
    const uint64_t T = h.T, seed = g.seed;
    const uint32_t graph_id = g.graph_id;
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K + 1));
    double *dA = (double *)malloc(sizeof(double) * (size_t)d);
    double *dB = (double *)malloc(sizeof(double) * (size_t)d * (size_t)(K + 1));
    for (uint64_t s = first; s < first + count; s++) {
        int32_t u;
        draw_tuple(&g, s, &u, &ids[0], &ids[1]);
        double eta = eta0 * (1.0 - (double)s / (double)T);
        for (int o = 2; o >= 1; o--) {
            if (!(orders & o)) continue;
            double *A = o == 2 ? U : U1, *B = o == 2 ? C : U1;
            sample_increments(&h, eta, A, B, u, ids, dA, dB);
            write_row_bf16(A, u, dA, d, seed, graph_id, s, (uint64_t)(16 * o), stream);
            for (int j = 0; j <= K; j++)
                write_row_bf16(B, ids[j], dB + (size_t)j * (size_t)d, d, seed, graph_id, s,
                               (uint64_t)(16 * o + 1 + j), stream);
        }
    }
    free(ids); free(dA); free(dB);
}

int or_train_bf16(const int32_t *src, const int32_t *dst, int64_t n, int64_t m,
                  const uint64_t *ethr, const int32_t *ealias,
                  const uint64_t *nthr, const int32_t *nalias,
                  uint64_t seed, uint32_t graph_id,
                  int d, int K, int orders, double eta0, double lambda, double alpha, uint64_t T,
                  double *U, double *C, double *U1, uint64_t first, uint64_t count,
                  uint64_t stream)
{
    if (d <= 0 || K < 0 || T == 0 || (orders & 3) == 0) return 1;
    if ((orders & 2) && (!U || !C)) return 1;
    if ((orders & 1) && !U1) return 1;
    or_graph g = {n, m, src, dst, ethr, ealias, nthr, nalias, seed, graph_id, K, NULL, NULL, 0};
    or_hyper h = {d, K, orders, eta0, lambda, alpha, T};
    train_range_bf16(&g, &h, U, C, U1, first, count, stream);
    return 0;
}

/* bfloat16 storage with the positive pairs of random walks (SEQ), as or_train_walk. */
int or_train_bf16_walk(const int32_t *src, const int32_t *dst, int64_t n, int64_t m,
                       const uint64_t *ethr, const int32_t *ealias,
                       const uint64_t *nthr, const int32_t *nalias,
                       const int64_t *off, const int32_t *nbr, const uint64_t *wthr, const int32_t *walias,
                       int L, int W, int64_t Bw,
                       uint64_t seed, uint32_t graph_id,
                       int d, int K, int orders, double eta0, double lambda, double alpha, uint64_t T,
                       double *U, double *C, double *U1, uint64_t first, uint64_t count,
                       uint64_t stream)
{
    if (d <= 0 || K < 0 || T == 0 || (orders & 3) == 0) return 1;
    if ((orders & 2) && (!U || !C)) return 1;
    if ((orders & 1) && !U1) return 1;
    or_walker wk = {n, m, src, dst, ethr, ealias, off, nbr, wthr, walias, seed, graph_id, L, W, Bw};
    if (!walker_ok(&wk)) return 1;
    const uint64_t per = (uint64_t)Bw * (uint64_t)walk_pairs_per_walk(L, W);
    or_hyper h = {d, K, orders, eta0, lambda, alpha, T};
    int32_t *pu = (int32_t *)malloc(sizeof(int32_t) * (size_t)per);
    int32_t *pv = (int32_t *)malloc(sizeof(int32_t) * (size_t)per);
    const uint64_t end = first + count;
    for (uint64_t s = first; s < end;) {
        uint64_t b = s / per, b0 = b * per, stop = b0 + per < end ? b0 + per : end;
        fill_walk_batch(&wk, b, pu, pv);
        or_graph g = {n, m, src, dst, ethr, ealias, nthr, nalias, seed, graph_id, K, pu, pv, b0};
        train_range_bf16(&g, &h, U, C, U1, s, stop - s, stream);
        s = stop;
    }
    free(pu); free(pv);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* A pre-generated pair pool (Sec. IV-C, the Augmented-Pair variant): walks    */
/* are run before training only until about sqrt(2 T) pairs are collected, and */
/* the training pairs are combinations of the collected ones.                  */
/*   Collected pairs: the first R pairs of the walk source in its sample order */
/*   (samples 0 .. R-1 above), (u_r, v_r).  R for a run of T samples is the     */
/*   least R >= 2 with R (R - 1) / 2 >= T (or_pool_size).                       */
/*   Expansion: the R^2 combinations (u_i, v_j) of one collected pair's first   */
/*   vertex with any collected pair's second vertex; i = j gives the collected  */
/*   pairs back, i != j the recombined ones (mostly not arcs of the graph).     */
/*   Sample s draws its positive pair from the expansion uniformly: with x0, x1 */
/*   the first two words of the Philox block an arc draw of sample s uses (key  */
/*   (seed, graph_id), counter (s, 0, 0, 0)), i = floor(x0 R / 2^64) and        */
/*   j = floor(x1 R / 2^64).  The negatives are drawn as for any sample.         */
/* ------------------------------------------------------------------------- */
uint64_t or_pool_size(uint64_t T)
{
    uint64_t R = 2;
    while ((u128)R * (u128)(R - 1) / 2 < (u128)T) R++;
    return R;
}

/* The R collected pairs: pu/pv[r] = the walk source's pair of sample r. */
static int pool_collect(const or_walker *wk, uint64_t R, int32_t *pu, int32_t *pv)
{
    const uint64_t per = (uint64_t)wk->Bw * (uint64_t)walk_pairs_per_walk(wk->L, wk->W);
    int32_t *bu = (int32_t *)malloc(sizeof(int32_t) * (size_t)per);
    int32_t *bv = (int32_t *)malloc(sizeof(int32_t) * (size_t)per);
    if (!bu || !bv) { free(bu); free(bv); return 1; }
    for (uint64_t b = 0; b * per < R; b++) {
        fill_walk_batch(wk, b, bu, bv);
        for (uint64_t i = 0; i < per && b * per + i < R; i++) {
            pu[b * per + i] = bu[i];
            pv[b * per + i] = bv[i];
        }
    }
    free(bu); free(bv);
    return 0;
}

static void pool_pair(const uint64_t *seed_gid, const int32_t *pu, const int32_t *pv, uint64_t R, uint64_t s,
                      int32_t *u, int32_t *v)
{
    uint64_t ctr[4] = {s, 0, 0, 0}, x[4];
    or_philox4x64_10(seed_gid[0], seed_gid[1], ctr, x);
    uint64_t i = (uint64_t)(((u128)x[0] * R) >> 64), j = (uint64_t)(((u128)x[1] * R) >> 64);
    *u = pu[i];
    *v = pv[j];
}

/* The collected pairs (pool_u/pool_v, R each) and the positive pairs of samples
 * [first, first + count) drawn from the pool of R pairs (u, v: count each; either pair of
 * outputs may be NULL). */
int or_pool_pairs(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                  const uint64_t *ethr, const int32_t *ealias,
                  const int64_t *off, const int32_t *nbr, const uint64_t *wthr, const int32_t *walias,
                  uint64_t seed, uint32_t graph_id, int L, int W, int64_t Bw, uint64_t R,
                  int32_t *pool_u, int32_t *pool_v, uint64_t first, uint64_t count, int32_t *u, int32_t *v)
{
    or_walker wk = {n, m, src, dst, ethr, ealias, off, nbr, wthr, walias, seed, graph_id, L, W, Bw};
    if (!walker_ok(&wk) || R < 1) return 1;
    int32_t *pu = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    int32_t *pv = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    if (!pu || !pv || pool_collect(&wk, R, pu, pv) != 0) { free(pu); free(pv); return 1; }
    if (pool_u && pool_v)
        for (uint64_t r = 0; r < R; r++) { pool_u[r] = pu[r]; pool_v[r] = pv[r]; }
    const uint64_t key[2] = {seed, (uint64_t)graph_id};
    if (u && v)
        for (uint64_t i = 0; i < count; i++) pool_pair(key, pu, pv, R, first + i, &u[i], &v[i]);
    free(pu); free(pv);
    return 0;
}

/* Training (or_train, or with bf16_stream >= 0 the bfloat16-storage SEQ run of
 * or_train_bf16 with that rounding stream) with positive pairs drawn from the pool of R
 * pairs.  SNAPSHOT batches may fall anywhere: the pairs of a range do not depend on how
 * it is cut. */
int or_train_pool(const int32_t *src, const int32_t *dst, int64_t n, int64_t m,
                  const uint64_t *ethr, const int32_t *ealias,
                  const uint64_t *nthr, const int32_t *nalias,
                  const int64_t *off, const int32_t *nbr, const uint64_t *wthr, const int32_t *walias,
                  int L, int W, int64_t Bw, uint64_t R,
                  uint64_t seed, uint32_t graph_id,
                  int d, int K, int orders, double eta0, double lambda, double alpha, uint64_t T,
                  double *U, double *C, double *U1,
                  uint64_t first, uint64_t count, int mode, uint64_t batch, int64_t bf16_stream)
{
    if (d <= 0 || K < 0 || T == 0 || (orders & 3) == 0) return 1;
    if ((orders & 2) && (!U || !C)) return 1;
    if ((orders & 1) && !U1) return 1;
    if (mode == 1 && batch == 0) return 1;
    if (bf16_stream >= 0 && mode != 0) return 1;
    or_walker wk = {n, m, src, dst, ethr, ealias, off, nbr, wthr, walias, seed, graph_id, L, W, Bw};
    if (!walker_ok(&wk) || R < 1) return 1;
    int32_t *cu = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    int32_t *cv = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    if (!cu || !cv || pool_collect(&wk, R, cu, cv) != 0) { free(cu); free(cv); return 1; }
    /* A SNAPSHOT batch must see all of its pairs at once: pieces are whole batches. */
    uint64_t piece = (uint64_t)1 << 20;
    if (mode == 1) piece = batch > piece ? batch : (piece / batch) * batch;
    int32_t *pu = (int32_t *)malloc(sizeof(int32_t) * (size_t)piece);
    int32_t *pv = (int32_t *)malloc(sizeof(int32_t) * (size_t)piece);
    const uint64_t key[2] = {seed, (uint64_t)graph_id};
    or_hyper h = {d, K, orders, eta0, lambda, alpha, T};
    int rc = (!pu || !pv) ? 1 : 0;
    const uint64_t end = first + count;
    for (uint64_t s = first; s < end && rc == 0;) {
        /* pieces start at multiples of `piece` (so at batch starts) */
        uint64_t p0 = (s / piece) * piece, stop = p0 + piece < end ? p0 + piece : end;
        for (uint64_t t = p0; t < stop; t++) pool_pair(key, cu, cv, R, t, &pu[t - p0], &pv[t - p0]);
        or_graph g = {n, m, src, dst, ethr, ealias, nthr, nalias, seed, graph_id, K, pu, pv, p0};
        if (bf16_stream >= 0)
            train_range_bf16(&g, &h, U, C, U1, s, stop - s, (uint64_t)bf16_stream);
        else
            rc = train_range(&g, &h, U, C, U1, s, stop - s, mode, batch);
        s = stop;
    }
    free(cu); free(cv); free(pu); free(pv);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Timing mode: the same per-sample rule in binary32, samples spread over     */
/* OpenMP threads with no locking (Hogwild).  Rows are read, increments are    */
/* computed from what was read, and the increments are added back; updates    */
/* that race are lost, as in any lock-free SGD.                                */
/* ------------------------------------------------------------------------- */
int or_train_hogwild_f32(const int32_t *src, const int32_t *dst, int64_t n, int64_t m,
                         const uint64_t *ethr, const int32_t *ealias,
                         const uint64_t *nthr, const int32_t *nalias,
                         uint64_t seed, uint32_t graph_id,
                         int d, int K, int orders, double eta0, double lambda, double alpha,
                         uint64_t T, float *U, float *C, float *U1,
                         uint64_t first, uint64_t count, int nthreads)
{
    if (d <= 0 || K < 0 || T == 0 || (orders & 3) == 0) return 1;
    if ((orders & 2) && (!U || !C)) return 1;
    if ((orders & 1) && !U1) return 1;
    or_graph g = {n, m, src, dst, ethr, ealias, nthr, nalias, seed, graph_id, K, NULL, NULL, 0};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K + 1));
        float *a = (float *)malloc(sizeof(float) * (size_t)d);
        float *dA = (float *)malloc(sizeof(float) * (size_t)d);
        float *b = (float *)malloc(sizeof(float) * (size_t)d * (size_t)(K + 1));
        float *dB = (float *)malloc(sizeof(float) * (size_t)d * (size_t)(K + 1));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < (int64_t)count; i++) {
            uint64_t s = first + (uint64_t)i;
            int32_t u;
            draw_tuple(&g, s, &u, &ids[0], &ids[1]);
            float eta = (float)(eta0 * (1.0 - (double)s / (double)T));
            float el = eta * (float)lambda, ea = eta * (float)alpha;
            for (int o = 2; o >= 1; o--) {
                if (!(orders & o)) continue;
                float *A = o == 2 ? U : U1, *B = o == 2 ? C : U1;
                for (int c = 0; c < d; c++) { a[c] = A[(int64_t)u * d + c]; dA[c] = 0.0f; }
                for (int j = 0; j <= K; j++)
                    for (int c = 0; c < d; c++) b[j * d + c] = B[(int64_t)ids[j] * d + c];
                for (int j = 0; j <= K; j++) {
                    float x = 0.0f;
                    for (int c = 0; c < d; c++) x += a[c] * b[j * d + c];
                    float sg = 1.0f / (1.0f + expf(-x));
                    float gj = j == 0 ? eta * (1.0f - sg) : -ea * sg;
                    for (int c = 0; c < d; c++) {
                        dA[c] += gj * b[j * d + c] - el * a[c];
                        dB[j * d + c] = gj * a[c] - el * b[j * d + c];
                    }
                }
                for (int c = 0; c < d; c++) A[(int64_t)u * d + c] += dA[c];
                for (int j = 0; j <= K; j++)
                    for (int c = 0; c < d; c++) B[(int64_t)ids[j] * d + c] += dB[j * d + c];
            }
        }
        free(ids); free(a); free(dA); free(b); free(dB);
    }
    return 0;
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Held-out link-prediction AUC (Mann-Whitney U statistic): the fraction of    */
/* (positive, negative) score pairs ranked correctly, ties counting one half.  */
/* Computed by sorting all scores and summing the mid-ranks of the positives.  */
/* ------------------------------------------------------------------------- */
typedef struct { double s; int pos; } scored;

static int cmp_scored(const void *x, const void *y)
{
    double a = ((const scored *)x)->s, b = ((const scored *)y)->s;
    return (a > b) - (a < b);
}

double or_auc(const double *pos, int64_t npos, const double *neg, int64_t nneg)
{
    if (npos <= 0 || nneg <= 0) return NAN;
    int64_t n = npos + nneg;
    scored *v = (scored *)malloc(sizeof(scored) * (size_t)n);
    for (int64_t i = 0; i < npos; i++) { v[i].s = pos[i]; v[i].pos = 1; }
    for (int64_t i = 0; i < nneg; i++) { v[npos + i].s = neg[i]; v[npos + i].pos = 0; }
    qsort(v, (size_t)n, sizeof(scored), cmp_scored);
    double rank_sum = 0.0;
    int64_t i = 0;
    while (i < n) {
        int64_t j = i;
        while (j + 1 < n && v[j + 1].s == v[i].s) j++;
        double mid = 0.5 * (double)(i + 1 + j + 1); /* ranks are 1-based */
        for (int64_t k = i; k <= j; k++)
            if (v[k].pos) rank_sum += mid;
        i = j + 1;
    }
    free(v);
    double u_stat = rank_sum - 0.5 * (double)npos * (double)(npos + 1);
    return u_stat / ((double)npos * (double)nneg);
}

/* Scores of pairs: A[u] . B[v] in binary64. */
void or_pair_scores(const double *A, const double *B, int d, const int32_t *u, const int32_t *v,
                    int64_t cnt, double *out)
{
    for (int64_t i = 0; i < cnt; i++) {
        double x = 0.0;
        for (int c = 0; c < d; c++) x += A[(int64_t)u[i] * d + c] * B[(int64_t)v[i] * d + c];
        out[i] = x;
    }
}
