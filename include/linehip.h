/*
 * linehip -- LINE-style edge-sampled SGD for graph embeddings on AMD Instinct MI355X
 * (gfx950).  C ABI.
 *
 * The method (NOMAD, arXiv 2604.09419, Sec. IV "Methods"):
 *   * a positive pair is an arc (u, v) drawn from the weight-normalised edge
 *     distribution (Algorithm 3, root-edge selection), or, after lh_walk_build, a pair
 *     of a random walk rooted at such an arc (Algorithms 2-3);
 *   * K negatives v- are drawn i.i.d. from q(v) proportional to d(v)^0.75, d the
 *     out-degree (Eq. (1));
 *   * per pair the signed gradient scalar is g = eta (1 - sigma(U[u].C[v])) for the
 *     positive and g = -eta alpha_neg sigma(U[u].C[v-]) for a negative (Algorithm 1,
 *     local updates), and LineUpdate / Eqs. (2)-(3) add g*C[.] - eta*lambda*U[u] to the
 *     vertex row and g*U0 - eta*lambda*C[.] to the context row;
 *   * a deterministic mode computes a batch's increments from the tables as they were
 *     at the batch start and sums them per row before applying (Eq. (4)).
 * First-order proximity (one table U1 at both ends) uses the same tuples.
 *
 * Conventions shared by every call
 *   - Pointers are plain addresses.  "device" means memory allocated on the handle's
 *     GPU (hipMalloc, or a torch tensor on that GPU); "host" means ordinary CPU memory.
 *   - The caller owns every buffer it passes in; the library never frees caller
 *     memory.  A handle owns only small host metadata and one int64 device status word.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Every call
 *     enqueues its work on the handle's stream; the calls whose comment says so
 *     (lh_set_graph, lh_build_alias, lh_export_alias, lh_tune, lh_check,
 *     lh_last_train_ms, lh_destroy and the batch calls that report results) synchronise
 *     it, the others return without waiting.
 *   - Argument errors are detected on the host before any GPU work and returned at
 *     once.  Errors in the graph (an ID >= n, a NaN or negative weight, a zero total
 *     weight) are found by lh_set_graph / lh_build_alias, which wait for their check and
 *     return them; an imported alias entry outside [0, N) is recorded on the device and
 *     reported by lh_check.
 *   - No call throws; every call returns an lh_status.  A handle must not be used
 *     from two threads at once; distinct handles are independent.
 *   - Tables are row-major [n x d] with rows of d elements (d % 8 == 0), binary32 or
 *     bfloat16 as lh_params.dtype says, and 16-byte-aligned base addresses.
 */
#ifndef LINEHIP_H
#define LINEHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LH_API __attribute__((visibility("default")))

typedef enum {
    LH_OK = 0,
    LH_ERR_INVALID_ARG = 1,      /* a null pointer, a size out of range, d % 8 != 0 ... */
    LH_ERR_OUT_OF_RANGE = 2,     /* device-detected: an arc endpoint >= n              */
    LH_ERR_ZERO_WEIGHT = 3,      /* device-detected: NaN/negative weight or zero total */
    LH_ERR_WORKSPACE_TOO_SMALL = 4,
    LH_ERR_NOT_BUILT = 5,        /* a call needs lh_bind / lh_set_graph / alias first   */
    LH_ERR_UNSUPPORTED = 6,      /* a parameter combination the library has no kernel for */
    LH_ERR_NO_DEVICE = 7,        /* no HIP device, or the device index is out of range  */
    LH_ERR_HIP = 8               /* a HIP runtime call failed; see lh_last_error       */
} lh_status;

enum { LH_FP32 = 0, LH_BF16 = 1 };
enum { LH_HOGWILD = 0, LH_SNAPSHOT = 1 };
enum { LH_ORDER1 = 1, LH_ORDER2 = 2, LH_ORDER12 = 3 };
enum { LH_TABLE_U = 0, LH_TABLE_C = 1, LH_TABLE_U1 = 2 };
enum { LH_ALIAS_EDGE = 0, LH_ALIAS_NEG = 1 };

typedef struct {
    int32_t d;          /* embedding width, d % 8 == 0, 8 <= d <= 512                    */
    int32_t K;          /* negatives per positive pair, 0 <= K <= 8 (Algorithm 1)        */
    int32_t orders;     /* LH_ORDER1 | LH_ORDER2 | LH_ORDER12                              */
    int32_t dtype;      /* LH_FP32 or LH_BF16 (tables; arithmetic is always binary32)     */
    double eta0;        /* initial step size eta (Sec. V-A: 0.025)                          */
    double lambda;      /* weight decay lambda of LineUpdate                                */
    double alpha_neg;   /* negative weight alpha_neg of Algorithm 1                         */
    uint64_t seed;      /* key word 0 of every Philox4x64-10 block                          */
    uint64_t total_samples; /* T: eta_s = eta0 (1 - s / T) for global sample index s     */
    int32_t mode;       /* LH_HOGWILD or LH_SNAPSHOT                                        */
    int32_t graph_id;   /* low 32 bits of key word 1 (one stream per graph)                 */
    int64_t batch;      /* SNAPSHOT batch B (samples [bB, (b+1)B) share one snapshot)      */
    double hot_rate;    /* HOGWILD: a row r is "hot" when W p_r >= hot_rate, p_r = the
                           probability that one sample touches r (from the degrees of the
                           last lh_build_alias), W = the launch's samples in flight
                           (unbounded when the tables fit in one XCD's L2: every touched
                           row is hot).  Hot rows take atomic increments, the others
                           coherent (system-scope) stores.  Rows of imported alias
                           tables are hot.  <= 0: every row atomic; >= 1e30: none.       */
    double max_conflicts; /* HOGWILD: the launch keeps F samples in flight with
                           F (2 + K) / n_active <= max_conflicts, n_active = nodes with an
                           arc, so that a row of average traffic has at most this many
                           concurrent writers (staleness bound).  <= 0: no cap.          */
    int32_t hot_shadow; /* HOGWILD with LH_BF16 tables: 0 = hot rows take packed bfloat16
                           atomic adds of SR(row + increment) - row, SR the stochastic
                           rounding a cold row is stored with (without a concurrent write
                           the result is SR(row + increment) exactly while |increment| <=
                           |row| / 2, else within one bfloat16 spacing); 1 = hot rows
                           accumulate in a binary32 shadow (one per table, up to
                           max(2^17, n/16) rows, in the workspace) for the duration of each
                           lh_train_steps launch and are rounded stochastically back into
                           the table after it.  Must be 0 or 1; ignored otherwise.         */
} lh_params;

typedef struct lh_handle lh_handle;
typedef struct lh_batch lh_batch;

/* Create a handle for device `device` after validating *p (the inputs of Algorithm 1:
 * d, K, lambda, eta, alpha_neg; Sec. V-A gives eta = 0.025).  Returns LH_ERR_NO_DEVICE
 * when no HIP device exists (so it can be probed without a GPU).  *h is owned by the
 * caller until lh_destroy. */
LH_API lh_status lh_create(lh_handle **h, const lh_params *p, int device);

/* Bytes of device memory the caller must provide for a graph with n nodes and m arcs
 * (the graph G = (V, E) of Algorithm 1's input): *persist for lh_bind (alias tables,
 * flags, SNAPSHOT buffers of the Eq. (4) batch) and *scratch for lh_build_alias (binary64
 * build arrays, free after that call's work has run).  Host-only; needs no device.
 * LH_ERR_INVALID_ARG for n < 1, n or m >= 2^31, or SNAPSHOT with 3 n >= 2^32. */
LH_API lh_status lh_workspace_size(const lh_params *p, int64_t n, int64_t m, size_t *persist,
                            size_t *scratch);

/* Attach caller memory: the embedding tables U and C that Algorithm 1 outputs (and U1
 * for first-order proximity).  workspace: device, >= *persist bytes from
 * lh_workspace_size for the n and m later given to lh_set_graph, 256-byte aligned.
 * tables[3]: device pointers to U, C, U1 ([n x d] each, lh_params.dtype, 16-byte
 * aligned), NULL for a table the orders do not use.  stream: the hipStream_t every later
 * call enqueues on.  The caller keeps ownership and must keep them alive while the handle
 * uses them.  LH_ERR_INVALID_ARG for a NULL or misaligned pointer. */
LH_API lh_status lh_bind(lh_handle *h, void *workspace, size_t bytes, void *const tables[3],
                  void *stream);

/* The graph G = (V, E) of Algorithm 1's input: n nodes, m arcs (src[a] -> dst[a],
 * weight w[a]); device arrays that must stay valid until lh_build_alias has returned.
 * An undirected edge is two arcs.  The
 * endpoints and weights are checked by a kernel and the call synchronises the stream:
 * LH_ERR_OUT_OF_RANGE for an endpoint outside [0, n), LH_ERR_ZERO_WEIGHT for a negative,
 * NaN or infinite weight; the handle then has no graph. */
LH_API lh_status lh_set_graph(lh_handle *h, int64_t n, int64_t m, const int32_t *src,
                       const int32_t *dst, const float *w);

/* Build the edge alias table over the m arcs (weights w: the root-edge distribution of
 * Algorithm 3) and the negative alias table over the n nodes (weights out-degree^0.75,
 * Eq. (1)) with the binary64 canonical chunked scan, and the per-node touch rates the Hogwild write path is chosen by.
 * scratch: device, >= *scratch bytes from lh_workspace_size, free once the call has
 * returned (it synchronises the stream).  LH_ERR_ZERO_WEIGHT when the arcs' total weight
 * is zero (or m == 0). */
LH_API lh_status lh_build_alias(lh_handle *h, void *scratch, size_t scratch_bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lh_build_alias without the scratch
 * argument.  The binary64 build arrays live in a 65 MiB array the library holds on each
 * GPU it runs on from its load to the end of the process, so the call allocates nothing;
 * it accepts graphs with n <= 2^21 and m <= 2^21 (LH_ERR_INVALID_ARG, before any GPU
 * work, for larger ones).  Results, synchronisation and errors as lh_build_alias.  Every
 * call on one GPU uses that GPU's one array: calls that overlap on one GPU (from two host
 * threads, or on two streams) race and must not be made. */
LH_API lh_status lh_build_alias_noalloc(lh_handle *h);

/* Replace (import) or copy out (export) one alias table, the encoding of the edge
 * distribution of Algorithm 3 (which = LH_ALIAS_EDGE, N = m) or of the negative
 * distribution of Eq. (1) (LH_ALIAS_NEG, N = n): column c keeps itself when a draw's
 * threshold word is below thr[c], else it yields alias[c].  thr uint64[N], alias int32[N],
 * both device, caller-owned.  Import checks the entries on the device (an alias outside
 * [0, N) is replaced by the column and reported by lh_check) and marks every row hot;
 * export synchronises the stream.  LH_ERR_NOT_BUILT when the table does not exist yet. */
LH_API lh_status lh_import_alias(lh_handle *h, int which, const uint64_t *thr, const int32_t *alias);
LH_API lh_status lh_export_alias(lh_handle *h, int which, uint64_t *thr, int32_t *alias);

/* Fill the bound tables with the initial values ("Initialize U and C" of Algorithm 1;
 * the paper gives no distribution, here both tables are uniform on [-0.5/d, 0.5/d)):
 * element (t, r, c) from Philox4x64-10 word c % 4 of key (seed, 2^32 | graph_id), counter
 * (r, c / 4, t, 0), value ((x >> 40) - 2^23) 2^-24 / d; bfloat16 tables take the
 * round-to-nearest-even of that value.  Enqueued; LH_ERR_NOT_BUILT before lh_set_graph. */
LH_API lh_status lh_init_embeddings(lh_handle *h);

/* The tuples of samples [first, first + count), as training draws them: the positive
 * pair (u, v) is an arc drawn proportionally to its weight (Algorithm 3, root-edge
 * selection) and the K negatives v- are drawn i.i.d. from q(v) ~ out-degree^0.75 (Eq. (1);
 * Algorithm 1 draws them without rejection).  Sample s slot j (0 = the arc, 1..K the
 * negatives) uses Philox4x64-10 key (seed, graph_id), counter (s, j, 0, 0).
 * Outputs (device, caller-owned): u[i], v[i] (int32, count each) and neg[i * K + k]
 * (int32, count * K; may be NULL when K = 0).  Enqueued, deterministic.
 * LH_ERR_NOT_BUILT before both alias tables exist; LH_ERR_INVALID_ARG for a NULL output,
 * a range that wraps past 2^64, or count >= 2^40. */
LH_API lh_status lh_sample(lh_handle *h, uint64_t first, uint64_t count, int32_t *u, int32_t *v,
                    int32_t *neg);

/* Train samples [first, first + count) in lh_params.mode (Algorithm 1, local updates):
 * per sample and order, x_j = A[u] . B[b_j] for the positive (j = 0) and the K negatives,
 * g_0 = eta_s (1 - sigma(x_0)), g_k = -eta_s alpha_neg sigma(x_k), then LineUpdate /
 * Eqs. (2)-(3): A[u] += sum_j (g_j B[b_j] - eta_s lambda A[u]) and
 * B[b_j] += g_j A[u] - eta_s lambda B[b_j], all from the rows as they were before the
 * sample; second order (A, B) = (U, C), first order A = B = U1, both on the same tuple.
 * eta_s = eta0 (1 - s / T).  HOGWILD applies samples concurrently without locks;
 * SNAPSHOT takes every increment of batch [bB, min((b+1)B, end)) against the tables at
 * the batch start and adds each row's ordered sum once (Eq. (4)), bit-reproducibly.
 * Enqueued.  LH_ERR_INVALID_ARG when first + count > T or (SNAPSHOT) first % batch != 0;
 * LH_ERR_NOT_BUILT before both alias tables exist. */
LH_API lh_status lh_train_steps(lh_handle *h, uint64_t first, uint64_t count);

/* (Execution only: the paper defines no tiling.)  Pick the Hogwild kernel
 * configuration (lanes per sample, 4-byte units per lane, workgroups per compute unit)
 * for this handle's shape by timing each candidate on samples [0, probe) with the step
 * size scaled to zero, so the tables are left as they were (binary32 and bfloat16).
 * cache_path (may be NULL) names a JSON file of earlier choices keyed by device, dtype,
 * d, K and orders; a hit skips the timing.  Synchronises. */
LH_API lh_status lh_tune(lh_handle *h, uint64_t probe, const char *cache_path);

/* The Hogwild kernel configuration in use: out[0] lanes per sample, out[1] 4-byte units
 * of a row per lane (one binary32 value or two bfloat16 values each), out[2] workgroups
 * per compute unit (host memory, 3 int32).  Until lh_set_kernel_config or lh_tune pins
 * one, lh_build_alias and lh_import_alias choose it from the degrees: bfloat16 handles
 * run two samples per wavefront when at most a tenth of the row touches would then fall
 * on hot rows, else one (imported tables, whose rows are all hot: one). */
LH_API lh_status lh_kernel_config(const lh_handle *h, int32_t out[3]);

/* Use configuration cfg (same layout as lh_kernel_config's out) for later Hogwild
 * launches, e.g. one found by the caller's own timing, and keep it across later alias
 * builds.  (lanes, units) must be one of
 * (16|32|64, 1 or 2), (2..64, 4), (4..64, 8) with lanes x units >= the row's units, and
 * 1 <= workgroups <= 64; else LH_ERR_INVALID_ARG and the configuration is unchanged. */
LH_API lh_status lh_set_kernel_config(lh_handle *h, const int32_t cfg[3]);

/* The output embeddings U and C of Algorithm 1 (and U1): copy rows [row0, row0 + rows)
 * of table t (LH_TABLE_*) to / from a binary32 device buffer [rows x d] (caller-owned);
 * bfloat16 tables convert (reads exactly, writes round to nearest even).  Enqueued.
 * LH_ERR_INVALID_ARG for a table the orders do not use or rows outside [0, n). */
LH_API lh_status lh_read_embeddings(lh_handle *h, int table, int64_t row0, int64_t rows, float *out);
LH_API lh_status lh_write_embeddings(lh_handle *h, int table, int64_t row0, int64_t rows,
                              const float *in);

/* (Error reporting, no counterpart in the paper.)  Synchronise the stream and report
 * device-side data errors (LH_ERR_OUT_OF_RANGE, LH_ERR_ZERO_WEIGHT) recorded since the
 * last lh_check, clearing them. */
LH_API lh_status lh_check(lh_handle *h);

/* (Measurement only.)  Kernel time of the last lh_train_steps call, in milliseconds,
 * measured with HIP events on the handle's stream (synchronises).  Returns 0 when
 * nothing was timed. */
LH_API lh_status lh_last_train_ms(lh_handle *h, double *ms);

LH_API const char *lh_status_string(lh_status s);
LH_API const char *lh_last_error(const lh_handle *h);
LH_API lh_status lh_destroy(lh_handle *h);

/* ---------------- Batched: many graphs in one persistent launch ----------------
 * (An execution extension: each graph is trained exactly as lh_train_steps trains it,
 * Algorithm 1 in HOGWILD mode; the paper trains one graph at a time.)
 * G handles (HOGWILD, second order, created and bound as above, alias tables built,
 * tables initialised) are trained together: one persistent kernel pulls (graph, chunk of
 * samples) items from a device work queue until every graph's [0, T_g) is done.
 * lh_batch_capture records the queue reset and the kernel into a hipGraph (captured on
 * the first handle's stream); lh_batch_launch replays it on `stream` (a hipStream_t as
 * void*, NULL = the first handle's stream), and lh_batch_run enqueues the same work
 * without a graph.  When `stream` is another stream, the launch waits for the work
 * already queued on the first handle's stream, and that stream waits for the launch, so
 * the handles' later calls see its result.  lh_batch_tune times the kernel variants
 * (lanes per sample, samples per item, grid size) on this batch and keeps the fastest;
 * cache_path (may be NULL) names a JSON file of earlier choices keyed by device and shape.
 * The batch object owns two small device buffers (the graph descriptors and the work
 * counters) and the hipGraph; lh_batch_destroy frees them.  It supports second-order
 * HOGWILD handles of one dtype with d <= 128; other mixes return LH_ERR_UNSUPPORTED. */
LH_API lh_status lh_batch_create(lh_batch **b, int G, lh_handle *const *graphs);
LH_API lh_status lh_batch_tune(lh_batch *b, const char *cache_path);
LH_API lh_status lh_batch_capture(lh_batch *b);
LH_API lh_status lh_batch_launch(lh_batch *b, void *stream);
LH_API lh_status lh_batch_run(lh_batch *b, void *stream);   /* same work as launch, without a graph */
LH_API lh_status lh_batch_last_ms(lh_batch *b, double *ms);
/* The batch's kernel configuration (host memory, 3 int64): out[0] the tile variant (0: one
 * 4-byte unit per lane for bfloat16 / four for binary32; 1: four / eight), out[1]
 * workgroups per compute unit, out[2] samples per work item; set by lh_batch_tune or the
 * defaults. */
LH_API lh_status lh_batch_config(const lh_batch *b, int64_t out[3]);
/* Samples trained per graph by the last launch/run (uint64[G], host; synchronises). */
LH_API lh_status lh_batch_done(lh_batch *b, uint64_t *done_per_graph);
LH_API lh_status lh_batch_destroy(lh_batch *b);

/* ---- Random-walk positive pairs (Sec. IV-B: Algorithm 2, RandomWalk, and Algorithm 3,
 * GeneratePairs; one GPU, so every vertex is local and no walk stops at a remote one).
 *
 * The walk graph is the undirected graph of the arcs: entry e < m is arc e forwards (tail
 * src[e], head dst[e]), entry m + e arc e backwards; both weigh w[e].  Row x, the
 * neighbourhood N(x), lists the entries with tail x in increasing entry index, and
 * discrete(N(x)) is an alias table over the row's weights built like the edge table
 * (binary64, canonical scans restarting at every row, items numbered within the row).
 * Walk k draws its root arc from the edge table with Philox4x64-10 key
 * (seed, 5 * 2^32 | graph_id), counter (k, 0, 0, 0): w_0 = its tail, w_1 = its head;
 * counter (k, t, 0, 0), t = 1 .. L - 2, draws w_{t+1} from row w_t.  A walk visits
 * L = walk_length vertices (Algorithm 2 counts visited vertices up to the walk length).
 * Its pairs are (w_i, w_{i+delta}), delta = 1 .. window - 1 (window 2: the consecutive
 * pairs Algorithm 2 collects), numbered p = sum_{delta' < delta} (L - delta') + i; P pairs
 * per walk.  Sample s = b Bw P + p Bw + j (Bw = walks_per_batch) takes pair p of walk
 * b Bw + j as its positive pair (u, v), so consecutive samples come from different walks
 * (Algorithm 3 shuffles a batch's pairs); its K negatives are drawn as before.
 *
 * lh_walk_size: bytes of device memory for a graph of n nodes and m arcs: *persist (row
 * offsets, row entries, and a pair buffer of whole walk batches, about 2^24 pairs) and
 * *scratch (build arrays, free once lh_walk_build has returned).  Host-only.
 * LH_ERR_INVALID_ARG unless 2 <= walk_length <= 4096, 2 <= window <= min(8, walk_length),
 * 1 <= walks_per_batch <= 2^24, walks_per_batch * P <= 2^27, m >= 1, 2m < 2^32. */
LH_API lh_status lh_walk_size(int64_t n, int64_t m, int32_t walk_length, int32_t window, int64_t walks_per_batch,
                              size_t *persist, size_t *scratch);

/* Build the walk rows of the handle's graph and switch its positive pairs to walks:
 * afterwards lh_train_steps (both modes) and lh_sample take (u, v) of sample s from the
 * walks as described above, generating each buffer fill of walks on the handle's stream
 * when a call first needs it.  persist and scratch: device, 256-byte aligned, at least
 * lh_walk_size's bytes; the caller owns both and keeps persist alive while the handle
 * uses the walks.  The graph arrays given to lh_set_graph must still be valid; the edge
 * table must exist (lh_build_alias).  Synchronises the stream.  LH_ERR_NOT_BUILT before
 * lh_build_alias; LH_ERR_INVALID_ARG for the ranges of lh_walk_size, or, in SNAPSHOT
 * mode, when the batch B does not divide walks_per_batch * P (a snapshot batch must lie
 * within one walk batch); LH_ERR_WORKSPACE_TOO_SMALL.  lh_bind and lh_set_graph drop the
 * walks; so does lh_walk_detach, returning to arc draws.  The batched launch does not
 * take handles with walks (LH_ERR_UNSUPPORTED), and lh_tune times arc draws. */
LH_API lh_status lh_walk_build(lh_handle *h, int32_t walk_length, int32_t window, int64_t walks_per_batch,
                               void *persist, size_t persist_bytes, void *scratch, size_t scratch_bytes);
LH_API lh_status lh_walk_detach(lh_handle *h);

/* The positive pairs (u, v) of samples [first, first + count) from the walks, exactly as
 * training takes them (the same buffer fills).  u, v: device int32[count], caller-owned.
 * Enqueued.  LH_ERR_NOT_BUILT before lh_walk_build; LH_ERR_INVALID_ARG for a NULL output
 * or a range that wraps past 2^64 or has count >= 2^40. */
LH_API lh_status lh_walk_pairs(lh_handle *h, uint64_t first, uint64_t count, int32_t *u, int32_t *v);

/* Copy out the walk rows (device, caller-owned): offsets int64[n + 1] (row x is entries
 * offsets[x] .. offsets[x + 1]), and per entry i the encoded discrete(N(x)): thr
 * uint64[2m], keep int32[2m] (the entry's head, kept when a draw's threshold word is
 * below thr[i]) and alias int32[2m] (the head of its alias entry otherwise).
 * Synchronises the stream.  LH_ERR_NOT_BUILT before lh_walk_build. */
LH_API lh_status lh_walk_export(lh_handle *h, int64_t *offsets, uint64_t *thr, int32_t *keep, int32_t *alias);

/* ---- A pre-generated pair pool (Sec. IV-C, the Augmented-Pair variant: walks run before
 * training only until about sqrt(2 T) pairs are collected, and the training pairs are
 * enumerated combinations of them, so sampling is decoupled from training).
 *
 * The pool's R collected pairs are the walk source's first R pairs (samples 0 .. R - 1
 * above), (u_r, v_r).  Its expansion is the R^2 combinations (u_i, v_j): i = j gives a
 * collected pair back, i != j a recombined one (mostly not an arc of the graph).  Sample
 * s draws its positive pair from the expansion uniformly with the Philox4x64-10 block an
 * arc draw of sample s would use (key (seed, graph_id), counter (s, 0, 0, 0)): with x0, x1
 * its first two words, i = floor(x0 R / 2^64) and j = floor(x1 R / 2^64).  Its K
 * negatives are drawn as before.
 *
 * lh_walk_pool_size: *pairs = the pool size for a run of total_samples samples, the least
 * R >= 2 with R (R - 1) / 2 >= total_samples.  Host-only.  LH_ERR_INVALID_ARG for a NULL
 * output or total_samples = 0. */
LH_API lh_status lh_walk_pool_size(uint64_t total_samples, uint64_t *pairs);

/* Switch the handle's positive pairs to a pool of `pairs` = R collected pairs (R >= 1;
 * 0 switches back to the walk pairs).  lh_train_steps (both modes) and lh_sample then
 * take their pairs from the pool.  The pool lives in the walk pair buffer (its first
 * fill, generated now on the handle's stream if it is not there); R may not exceed that
 * buffer's pairs (LH_ERR_OUT_OF_RANGE: about 2^24, enough for total_samples up to about
 * 1.4 10^14).  Enqueued.  LH_ERR_NOT_BUILT before lh_walk_build.  While a pool is on,
 * lh_walk_pairs returns LH_ERR_UNSUPPORTED (lh_sample gives the pool's pairs);
 * lh_walk_build and lh_walk_detach end the pool. */
LH_API lh_status lh_walk_pool(lh_handle *h, uint64_t pairs);

/* Number of exported entry points (for load checks) and their names. */
LH_API int lh_abi_symbol_count(void);
LH_API const char *lh_abi_symbol_name(int i);

#ifdef __cplusplus
}
#endif
#endif /* LINEHIP_H */
