/*
 * kc.h -- exact and colour-sampled k-clique counting on one AMD Instinct MI355X.
 *
 * The method is the one of Finocchi, Finocchi & Fusco, "Clique counting in
 * MapReduce: theory and experiments" (arXiv 1403.0734):
 *   - nodes are totally ordered by (degree, label) (Section 2);
 *   - every node u keeps its high-neighbourhood Gamma+(u), the neighbours above
 *     it in that order (Section 2; Algorithm 1, round 1);
 *   - every k-clique is counted once, by its smallest node u, as a (k-1)-clique
 *     of the subgraph G+(u) induced by Gamma+(u) (Section 3, Algorithm 1 rounds
 *     2-3, Theorem 1);
 *   - colour sampling (cFFF_k, Section 6) keeps only monochromatic pairs of each
 *     Gamma+(u) and scales the raw count back up.
 *
 * Conventions for every entry point:
 *   - Plain C types only.  Every call returns kc_status: KC_OK (0) or a negative
 *     error code; kc_status_str() gives a message (with the last HIP error text
 *     for KC_EDEVICE).
 *   - Node ids are uint32 in [0, n).  Per-node outputs are indexed by these
 *     original ids.
 *   - A kc_graph handle owns every device buffer it allocates; it is freed by
 *     kc_graph_destroy().  A handle is used by one host thread at a time.
 *   - All work runs on the HIP stream bound at creation (NULL = the default
 *     stream).  Calls that return host scalars synchronise that stream before
 *     returning; calls that write device arrays are ordered on the stream and
 *     have completed when the call returns.
 *   - Counts are exact uint64.  A total that does not fit in 64 bits is never
 *     wrapped: the call returns KC_EOVERFLOW.
 *   - Sizes: n < 2^32 and m_in < 2^31 (the canonicalisation sorts 2*m_in keys).
 */
#ifndef KC_H
#define KC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kc_status;
typedef struct kc_graph kc_graph;

enum {
    KC_OK = 0,
    KC_EINVAL = -1,    /* bad argument: null pointer, id >= n, k or c out of range */
    KC_ESTATE = -2,    /* call out of order, e.g. counting before kc_orient */
    KC_ENOMEM = -3,    /* device or host allocation failed */
    KC_EOVERFLOW = -4, /* an exact count does not fit in uint64 */
    KC_EDEVICE = -5    /* a HIP call failed */
};

/* Colour schemes for kc_count_colored. */
enum {
    KC_COLOR_PER_ROOT = 0, /* cFFF_k (Section 6): each root colours its own Gamma+(u);
                              a k-clique survives with probability c^-(k-2) */
    KC_COLOR_GLOBAL = 1    /* one colouring of all nodes; a k-clique survives when all
                              k nodes share a colour, probability c^-(k-1) */
};

/* Scheduling policies (kc_set_schedule); counts never depend on them. */
enum {
    KC_SCHED_DEGREE = 0,  /* plain degree binning: tier by out-degree, queue ordered by out-degree
                             descending, every root one work item */
    KC_SCHED_LEARNED = 1, /* from k = 5, the workgroup tier's roots ordered and split over several
                             work items (Section 7) by an MLP's predicted per-root work, and
                             one-wave roots with large predicted work promoted to the workgroup
                             tier; the degree queue below k = 5 */
    KC_SCHED_EDGES = 2    /* the default: as the degree policy, but from k = 5 the workgroup tier's
                             roots ordered and split by an estimate from the edges of G+(u) (c^1.5/d^2
                             for c edges and d nodes), known once the handle has staged G+(u) */
};

/* Parameters of the scheduler MLP (8 -> 32 -> 32 -> 1, ReLU, fp32), in this order:
 * W1[32][8], b1[32], W2[32][32], b2[32], w3[32], b3. */
#define KC_MLP_PARAMS 1377

/* Largest clique size the counting kernels accept. */
#define KC_KMAX 10

typedef struct {
    uint64_t raw;              /* cliques that survived the colouring (exact integer) */
    double estimate;           /* raw * c^e rounded to nearest double, e = k-2 or k-1 */
    uint64_t estimate_u64;     /* raw * c^e when it fits in 64 bits, else 0 */
    int32_t estimate_fits_u64; /* 1 if estimate_u64 is exact */
    int32_t scale_exponent;    /* e */
} kc_estimate;

/* Ingest (Section 2: the input is an edge set; degrees are computed here).
 * src[i], dst[i] (i < m_in) are the endpoints of edge i.  Self-loops are dropped,
 * each undirected pair is kept once, and d(u) is the degree in that simple graph.
 * src/dst are device pointers if src_on_device != 0, else host pointers; they are
 * read during the call only (the handle keeps its own copy).  hip_stream is a
 * hipStream_t or NULL.  Errors: KC_EINVAL for null pointers, n == 0, an id >= n or
 * m_in >= 2^31; KC_ENOMEM; KC_EDEVICE. */
kc_status kc_graph_create(const uint32_t *src, const uint32_t *dst, uint64_t m_in, uint32_t n,
                          int32_t src_on_device, void *hip_stream, kc_graph **out);

/* Orientation (Section 2 total order; Algorithm 1, round 1): nodes are relabelled
 * by their position in the (degree, label) order and every edge is kept once,
 * from its smaller to its larger endpoint; each out-list is sorted.  Idempotent. */
kc_status kc_orient(kc_graph *g);

/* Exact q_k (Section 3, Theorem 1) for 1 <= k <= KC_KMAX: q_1 = n, q_2 = m, and for
 * k >= 3 the sum over u of the (k-1)-cliques of G+(u).  The first count on a handle
 * stages every G+(u) into a device cache kept by the handle (about 8 bytes per edge
 * plus the bitmaps of roots above the one-wave limit; not kept when it would take
 * more than half the free device memory, or with KC_STAGE_CACHE=0); later counts of
 * any k and either colouring read it.  The staging pass itself yields q_3.  From
 * k = 7 the handle runs its one-wave tier on a second stream of its own (created on
 * first use, joined back before the call returns, destroyed with the handle).
 * KC_ESTATE if not oriented; KC_EOVERFLOW if q_k >= 2^64. */
kc_status kc_count(const kc_graph *g, int32_t k, uint64_t *q_out);

/* Colour-sampled estimate (Section 6, cFFF_k) for 3 <= k <= KC_KMAX and c >= 1.
 * Colours depend on the original ids and on seed:
 *   h = mix64(seed ^ mix64((u << 32) | x))  (per-root scheme, x in Gamma+(u)),
 *   h = mix64(seed ^ mix64(x))              (global scheme),
 *   colour = ((h >> 32) * c) >> 32,
 * with mix64 the SplitMix64 finaliser.  c == 1 gives raw == q_k. */
kc_status kc_count_colored(const kc_graph *g, int32_t k, uint32_t c, uint64_t seed, int32_t scheme,
                           kc_estimate *out);

/* Plain pair-sampled estimate (Section 6, plain pair sampling, FFF_k(p)) for
 * 3 <= k <= KC_KMAX and 0 < p <= 1: every pair {x, y} of Gamma+(u) joined by an
 * edge is kept independently per root u; raw = sum over u of the (k-1)-cliques of
 * the sampled G+(u); estimate = raw / p'^e with e = C(k-1, 2) (scale_exponent) and
 * p' = t / 2^32 the exact keep probability, t = floor(p 2^32).  The pair (x, y), x
 * before y in the order, is kept iff (H2 >> 32) < t with
 *   H2 = mix64(mix64(seed ^ mix64((u << 32) | x)) ^ mix64(y))  (original ids).
 * estimate_u64 is exact (and set) only for p = 1, where raw == q_k.  Counts a masked
 * copy of the handle's staged cache: KC_ENOMEM when the cache is not kept. */
kc_status kc_count_pair_sampled(const kc_graph *g, int32_t k, double p, uint64_t seed, kc_estimate *out);

/* Per-root counts q_{u,k-1} (Section 3: the count the reducer for u emits) into the
 * caller's device array dev_counts[n], indexed by original id; optionally the
 * per-root intersection work into dev_work[n] (may be NULL): the number of
 * l-cliques of G+(u) for l = 1 .. k-2, i.e. the neighbourhood intersections an
 * unpruned depth-first count performs.  3 <= k <= KC_KMAX. */
kc_status kc_count_per_root(const kc_graph *g, int32_t k, uint64_t *dev_counts, uint64_t *dev_work);

/* Per-node clique-membership counts (Section 3, the remark after the round-3
 * reducers: a reducer can report, per node, the cliques of its sub-problem that
 * contain it): dev_counts[v] = the number of k-cliques that contain v, for every
 * node v, indexed by original id, in the caller's device array of n uint64
 * (overwritten; the call returns when it is written).  Sums to k * q_k.
 * 1 <= k <= KC_KMAX (k = 1: 1 each; k = 2: the degree).  For k >= 3 the local
 * graphs are read from the handle's staged G+(u) cache (built here if absent):
 * KC_ENOMEM when the cache is not kept; KC_EOVERFLOW when a count needs more than
 * 64 bits; KC_EINVAL when the largest out-degree needs more LDS per wave than a
 * workgroup has ((k - 2) * ceil(d / 64) * 8 bytes). */
kc_status kc_count_per_node(const kc_graph *g, int32_t k, uint64_t *dev_counts);

/* Exact q_k (3 <= k <= KC_KMAX) of num graphs at once; q_out[i] is the count of gs[i].
 * The graphs are laid side by side on the device as one disjoint union and counted
 * by the persistent tier kernels from one work queue (ordered by tier, graph and
 * out-degree).  The plan built on the first call stages every G+(u) of the union
 * once (device memory of about 8 bytes per edge plus the larger roots' bitmaps,
 * held until a different batch is planned or one of its handles is destroyed; not
 * kept, and staged on every replay, when it would take more than half the free
 * device memory), and captures the from-cache count launches in a HIP graph that is
 * replayed when the same graphs (same handles) are counted again at the same k.
 * Every graph must be oriented, on the same device and bound to the same stream;
 * num <= 65536. */
kc_status kc_count_batch(kc_graph *const *gs, uint32_t num, int32_t k, uint64_t *q_out);

/* Exact q_k (3 <= k <= KC_KMAX) with no device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The same kernels and result as kc_count, on a handle that an
 * earlier kc_count (any k >= 3) has prepared; KC_ESTATE otherwise.  It counts from
 * the handle's staged cache when kept, and always with the degree queue (counts do
 * not depend on the schedule).
 *   - dev_out: caller device memory of two uint64: [0] q_k, [1] 1 if q_k >= 2^64
 *     (then [0] is not the count), else 0.
 *   - Enqueued on the handle's stream and not waited for: dev_out holds the result
 *     once the stream has reached this call.  Nothing is read back to the host.
 *   - Scratch: one 64 MiB device array per GPU, held from the first call on that
 *     GPU until the process ends.  KC_EINVAL when a root's scratch-tier slice does
 *     not fit in it (out-degrees above about 32000).
 *   - Every call on a GPU shares that array: calls that overlap on one GPU (other
 *     streams, other threads) race. */
kc_status kc_count_noalloc(const kc_graph *g, int32_t k, uint64_t *dev_out);

/* Scheduling policy for later counts.  For KC_SCHED_LEARNED, weights_path names a
 * weight file written by kc_train_schedule (NULL keeps the weights already loaded). */
kc_status kc_set_schedule(kc_graph *g, int32_t policy, const char *weights_path);

/* The scheduler MLP's predictions with the handle's loaded weights (KC_ESTATE
 * without): dev_pred[n] (device, by original id) = the predicted log(1 + W(u, k)),
 * W the per-root work kc_count_per_root reports, for every root with out-degree
 * >= k-1 (0 for the others); dev_feat[n][8] (device, may be NULL) = the eight raw
 * features it read: log1p d+(u), log1p sum of d+ over Gamma+(u), log1p max d+ over
 * Gamma+(u), log1p d(u), log1p e+(u), e+(u) / C(d+(u), 2), k / 10, and
 * log C(d+(u), k-1) + C(k-1, 2) log(e+(u) / C(d+(u), 2)) clamped to [-10, 60] (-10
 * when undefined), with e+(u) the edges of G+(u).  3 <= k <= KC_KMAX. */
kc_status kc_predict_work(const kc_graph *g, int32_t k, float *dev_pred, float *dev_feat);

/* One training step of the scheduler MLP, the kernels kc_train_schedule runs per
 * mini-batch: the gradient of 0.5 * mean over the count samples of (y - t)^2, with
 * y the MLP's output for the standardised features dev_x[count][8] and dev_t[count]
 * the standardised labels, then one Adam update (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias correction at `step` >= 1) of dev_params[KC_MLP_PARAMS] with its moment
 * vectors dev_adam_m, dev_adam_v (same size; zero before step 1).  dev_grad
 * (KC_MLP_PARAMS, may be NULL) receives the gradient; *loss (host, may be NULL) the
 * batch loss before the update.  All device pointers; runs on hip_stream (NULL = the
 * default stream) and has completed when the call returns. */
kc_status kc_mlp_step(float *dev_params, float *dev_adam_m, float *dev_adam_v, int32_t step, float lr,
                      const float *dev_x, const float *dev_t, uint32_t count, float *dev_grad, float *loss,
                      void *hip_stream);

/* Train the scheduler's MLP (8 features -> 32 -> 32 -> 1, ReLU, fp32) on the GPU
 * to predict log(1 + per-root work) (the work kc_count_per_root reports) of every
 * root with at least k'-1 high neighbours, for every clique size k' = 4..k, over
 * the given oriented graphs: `epochs` passes of mini-batch Adam from a seeded
 * initialisation.  Writes the weights and the feature normalisation to
 * weights_path; *final_loss (may be NULL) is the last epoch's mean squared error
 * of the standardised label.  4 <= k <= KC_KMAX. */
kc_status kc_train_schedule(kc_graph *const *gs, uint32_t num, int32_t k, int32_t epochs, uint64_t seed,
                            const char *weights_path, float *final_loss);

/* Launch tunables (process-wide; counts never depend on them). */
typedef struct {
    int32_t wave_dmax;          /* roots with out-degree <= wave_dmax (1..64) go to the one-wave tier */
    int32_t wg_blocks_per_cu;   /* workgroup-tier blocks per CU, 0 = as many as LDS allows (0..8) */
    int32_t wave_blocks_per_cu; /* persistent wave-tier blocks of 4 waves per CU (1..16) */
    int32_t queue_chunk_div;    /* queue chunk = roots / (workers * queue_chunk_div) (1..64) */
    int32_t wg_dmax;            /* roots above wave_dmax with out-degree <= wg_dmax keep their bitmap in
                                   LDS (workgroup tier), larger ones in a global-memory slice (scratch
                                   tier); 0 = as large as LDS allows, else 64..65535 (lowered to the
                                   LDS limit when above it) */
    int32_t local_bits;         /* width of the local graphs that candidate sets of workgroup-tier roots
                                   are compacted into, in nodes: 64 (one word per row) or 128 (two
                                   words; used from k = 6); 0 = 128 */
    int32_t wg_waves;           /* waves per workgroup-tier block: 4, 8 or 16, or 0 = per launch, the
                                   shape that keeps the most waves resident (LDS, registers) */
} kc_tuning;

/* Set the tunables (NULL restores the defaults 64, 0, 8, 8, 0, 128, 0); KC_EINVAL outside the ranges. */
kc_status kc_set_tuning(const kc_tuning *t);
kc_status kc_get_tuning(kc_tuning *t);

/* Autotuner: times kc_count_batch(gs, num, k) over a grid of tunables, keeps the
 * fastest and applies it.  Results are cached in the JSON file cache_path (may be
 * NULL) under a key of the device architecture and the batch's size and k; a
 * cached entry is applied without timing.  *best (may be NULL) receives it. */
kc_status kc_autotune(kc_graph *const *gs, uint32_t num, int32_t k, const char *cache_path, kc_tuning *best);

kc_status kc_graph_info(const kc_graph *g, uint32_t *n, uint64_t *m, uint32_t *max_outdeg);

/* Copies of the handle's device arrays into caller device memory:
 * the simple graph's CSR (row_ptr[n+1], col[2m]) and degrees deg[n]; the oriented
 * CSR in rank space (optr[n+1], ocol[m]) and rank2id[n].  Any pointer may be NULL. */
kc_status kc_get_csr(const kc_graph *g, uint64_t *row_ptr, uint32_t *col, uint32_t *deg);
kc_status kc_get_oriented(const kc_graph *g, uint64_t *optr, uint32_t *ocol, uint32_t *rank2id);

/* Stage timings of the last count on this handle (milliseconds, HIP events on the
 * bound stream): queue building, the counting kernels, and their sum; and each
 * tier kernel alone (one-wave, workgroup, scratch; 0 for an empty tier). */
kc_status kc_last_timings(const kc_graph *g, float *ms_schedule, float *ms_count, float *ms_total);
kc_status kc_last_tier_timings(const kc_graph *g, float *ms_wave, float *ms_workgroup, float *ms_scratch);
/* The tier kernels of the staging pass (G+(u) into the handle's cache) of the last
 * count that staged: one-wave, workgroup and scratch kernels (milliseconds, HIP
 * events on the bound stream; 0 for an empty tier). */
kc_status kc_last_stage_timings(const kc_graph *g, float *ms_wave, float *ms_workgroup, float *ms_scratch);

void kc_graph_destroy(kc_graph *g);
const char *kc_status_str(kc_status s);

#ifdef __cplusplus
}
#endif

#endif /* KC_H */
