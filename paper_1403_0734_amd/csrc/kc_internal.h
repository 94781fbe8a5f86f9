// Internal declarations of libkc (gfx950, wave64).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kc.h"

// ----------------------------------------------------------------------------
// Error plumbing
kc_status kc_fail(kc_status s, const char *fmt, ...);
kc_status kc_hip_fail(hipError_t e, const char *what, const char *file, int line);

#define KC_HIP(x)                                                      \
    do {                                                               \
        hipError_t kc_e_ = (x);                                        \
        if (kc_e_ != hipSuccess) return kc_hip_fail(kc_e_, #x, __FILE__, __LINE__); \
    } while (0)

#define KC_TRY(x)                        \
    do {                                 \
        kc_status kc_s_ = (x);           \
        if (kc_s_ != KC_OK) return kc_s_; \
    } while (0)

// ----------------------------------------------------------------------------
// Device memory from the library's caching allocator (kc_alloc.hip): a block
// freed on stream s is reused by later work on s at once, and by any stream
// after kc_sync(s).
kc_status kc_cache_alloc(void **p, size_t bytes, hipStream_t s);
void kc_cache_free(void *p, hipStream_t s);
// Host synchronisation of s; s's freed blocks become reusable on any stream.
kc_status kc_sync(hipStream_t s);

// Temporary buffer of one call, freed on its stream when it goes out of scope.
struct kc_tmp {
    void *p = nullptr;
    hipStream_t s = nullptr;
    kc_tmp() = default;
    kc_tmp(const kc_tmp &) = delete;
    kc_tmp &operator=(const kc_tmp &) = delete;
    ~kc_tmp() { kc_cache_free(p, s); }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};
kc_status kc_tmp_alloc(kc_tmp &t, size_t bytes, hipStream_t s);
// Allocation owned by a handle (released with kc_cache_free on its stream).
kc_status kc_dev_alloc(void **p, size_t bytes, hipStream_t s);
// A small pinned host buffer owned by the calling thread (512 bytes).
uint64_t *kc_pinned_scratch();
// A pinned host buffer of at least `bytes` owned by the calling thread (grown on
// demand; the previous contents and pointer are invalid after a larger request).
void *kc_pinned_buffer(size_t bytes);

// ----------------------------------------------------------------------------
// The handle.
struct kc_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t n = 0;
    uint64_t m_in = 0;
    uint64_t m = 0;       // undirected edges of the simple graph
    int idbits = 1;       // bits that hold any id in [0, n)

    // simple graph: degrees, unique edges, symmetric CSR (built on request)
    uint64_t *rowptr = nullptr;  // n + 1
    uint32_t *col = nullptr;     // 2m
    uint32_t *deg = nullptr;     // n
    uint64_t *ukeys = nullptr;   // m sorted unique edges (min << idbits | max)

    // orientation, rank space
    int oriented = 0;
    uint64_t *optr = nullptr;     // n + 1
    uint32_t *ocol = nullptr;     // m
    uint32_t *rank2id = nullptr;  // n
    uint32_t *id2rank = nullptr;  // n
    uint32_t max_outdeg = 0;

    // schedule
    int policy = KC_SCHED_EDGES;
    float *mlp = nullptr;   // device weights (KC_MLP_PARAMS floats + normalisation)
    int mlp_loaded = 0;
    uint64_t *tri = nullptr;  // per-root edges of G+(u) by original id (scheduler feature), cached
    float *feat = nullptr;    // scheduler features that do not depend on k, cached (rank order)
    uint32_t feat_upto = 0;   // features are valid for the first feat_upto roots of the degree queue
    int feat_dqwd = -1;       // ... built with this wave-tier limit
    uint64_t mlp_serial = 0;  // bumped on every weight load
    // learned queue of each clique size, built once per (weights, tier limits)
    struct LearnedQueue {
        int ready = 0, wd = 0;
        uint32_t dcap = 0;
        uint64_t wserial = 0;
        uint32_t *queue = nullptr;   // scratch, workgroup, one-wave tier (with the degree queue's tail)
        uint64_t *items = nullptr;   // workgroup tier as split items (k >= 5)
        uint32_t item_count = 0;
        bool l2 = false;             // the items include two-level items
        // with dsplit > 0: items cover the roots above out-degree dsplit, items2 the rest
        uint32_t dsplit = 0;
        uint64_t *items2 = nullptr;
        uint32_t item_count2 = 0;
        bool l2b = false;
        uint32_t count[3] = {0, 0, 0}, max_d[3] = {0, 0, 0};  // kc_queue order: wave, workgroup, scratch
    } lq[KC_KMAX + 1];

    // small result area on the device: [0] total, [1] overflow flag, [2..] cursors
    uint64_t *d_res = nullptr;

    // degree-ordered work queue, built once per graph: roots with out-degree
    // above 64 first, then the rest down to out-degree 2, each part by
    // out-degree descending; plus the out-degree histogram on the host
    int dq_ready = 0;
    int dq_wd = 64;  // wave-tier out-degree limit the queue was split at
    uint32_t *dq = nullptr;
    uint32_t dq_wide = 0, dq_narrow = 0;
    uint64_t *dq_hist = nullptr;  // host, max_outdeg + 1 entries

    // Staged local graphs G+(u), built by the first count and read by later ones:
    // roots with out-degree <= stage_wd keep one 64-bit row per node of
    // Gamma+(u) at lrows[optr[u] + i] (bit j: a_j in Gamma+(a_i)); larger roots
    // keep their packed upper-triangular bitmap at wbits + woff[u].
    int staged = 0;  // 1 built, -1 not kept (memory), 0 not yet
    int stage_wd = 0;
    uint64_t stage_words = 0;  // words at wbits
    uint64_t *lrows = nullptr, *wbits = nullptr, *woff = nullptr;
    const uint64_t *wbits_raw = nullptr;  // set in a masked view: the bitmaps as staged

    // Workgroup-tier items for counts from k = 5 on (degree policy, staged
    // handles): the tier's roots by edges of G+(u), heaviest first, the heaviest
    // split over several items (rank << 32 | part << 16 | parts).  Built for the
    // tier span [wq_first, wq_first + wq_roots) of the degree queue.
    int wq_ready = 0;
    uint32_t wq_first = 0, wq_roots = 0, wq_count = 0;
    uint64_t *wq = nullptr;
    bool wq_l2 = false;          // wq holds two-level items
    // With wq_dsplit > 0, wq holds the items of the tier's roots above out-degree
    // wq_dsplit and wq2 those of the others (each launched with an arena of its own size).
    uint32_t wq_dsplit = 0;
    uint64_t *wq2 = nullptr;
    uint32_t wq2_count = 0;
    bool wq2_l2 = false;
    uint32_t *wedges = nullptr;  // edges of G+(u) by rank, written when staging (roots above stage_wd)

    uint64_t serial = 0;  // unique per handle (batch plans are keyed by it)
    hipEvent_t ev[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // second stream of the handle: the workgroup tier's large roots run on it beside
    // its small ones (fork / join events, no timing; created on first use)
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    float t_schedule = 0.f, t_count = 0.f, t_total = 0.f;
    float t_tier[3] = {0.f, 0.f, 0.f};  // wave, workgroup, scratch kernels of the last count
    hipEvent_t sev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // around the staging tiers
    float t_stage_tier[3] = {0.f, 0.f, 0.f};  // wave, workgroup, scratch kernels of the last staging pass
};

// ----------------------------------------------------------------------------
// Device-wide primitives (kc_prims.hip)
kc_status kc_scan_excl_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *d_total, hipStream_t s);
kc_status kc_scan_excl_u64(const uint64_t *in, uint64_t *out, size_t n, uint64_t *d_total, hipStream_t s);
// Stable LSD radix sort of 64-bit keys on bits [bit_lo, bit_hi).  tmp is a
// same-sized buffer.  The sorted keys end in keys, or, when `sorted` is given,
// in whichever of the two buffers the last pass wrote (*sorted), with no copy.
kc_status kc_radix_sort_u64(uint64_t *keys, uint64_t *tmp, size_t n, int bit_lo, int bit_hi, hipStream_t s,
                            uint64_t **sorted = nullptr);

// Ingest and orientation (kc_graph.hip)
kc_status kc_canonicalise(kc_graph *g, const uint32_t *d_src, const uint32_t *d_dst);
kc_status kc_orient_impl(kc_graph *g);
kc_status kc_build_csr(kc_graph *g);

// Counting (kc_count.hip)
struct kc_count_args {
    int k = 3;
    int colored = 0;
    uint32_t c = 1;
    uint64_t seed = 0;
    int scheme = KC_COLOR_PER_ROOT;
    uint64_t *per_root = nullptr;  // device [n] by original id, optional
    int policy = KC_SCHED_DEGREE;
    int cached = 0;  // count from the handle's staged G+(u) cache
    int store = 0;   // stage G+(u) into the cache, count nothing
    int sampled = 0;      // plain pair sampling: count a masked copy of the cache
    uint64_t pair_t = 0;  // keep threshold on the pair hash's high 32 bits (2^32 keeps all)
};
kc_status kc_count_impl(const kc_graph *g, const kc_count_args &a, uint64_t *total, int *overflow);
struct kc_queue;
uint32_t kc_lds_dcap(int device, int k);
// Four-wave workgroup blocks per CU that LDS allows for an arena holding out-degree d.
uint32_t kc_wg_blocks_per_cu(int device, int k, uint32_t d);
kc_status kc_count_scratch(const kc_graph *g, const kc_queue &q, int k, kc_tmp &gscr, size_t &slice_words,
                           uint32_t &blocks);
// tier_ev (may be null): 6 events: [0] before the scratch tier, [1] after it (before
// the workgroup tier), [2] after the workgroup tier, [3] after every tier,
// [4] [5] around the one-wave tier.
kc_status kc_count_launch(const kc_graph *g, const kc_queue &q, const kc_count_args &a, uint64_t *res,
                          unsigned long long *gtotals, uint32_t ngraphs, const uint32_t *graph_of, uint64_t *gscratch,
                          size_t slice_words, uint32_t scratch_blocks, hipStream_t s,
                          hipEvent_t *tier_ev = nullptr, bool use_side = false);

// Stage every root's G+(u) into the handle's cache (one-wave tier split at wd); the
// handle is left uncached (staged = -1) when the cache would not fit.
kc_status kc_stage(kc_graph *g, int wd);
// Stage the G+(u) of the roots in queue q of graph g into caches allocated here
// (rows for roots with out-degree <= wd, packed bitmaps above), enqueued on g's
// stream with a result block the caller owns (KC_RES_WORDS words); cached is false
// (and nothing is staged) when the caches would take more than half the free memory
// or a workgroup-tier root does not fit the staging kernels' arena.
kc_status kc_stage_queue(const kc_graph *g, const kc_queue &q, int wd, uint64_t *res, kc_tmp &lrows, kc_tmp &wbits,
                         kc_tmp &woff, bool &cached);

// Drop a cached batch plan that refers to the handle with this serial.
void kc_batch_forget(uint64_t serial);

// Launch tunables (process-wide; set by kc_set_tuning or kc_autotune).
struct kc_tuning_t {
    int wave_dmax = 64;          // roots with out-degree <= this go to the wave tier
    int wg_blocks_per_cu = 0;    // 0: as many as LDS allows (at most 8)
    int wave_blocks_per_cu = 8;  // persistent wave-tier blocks per CU
    int chunk_div = 8;           // queue chunk = roots / (workers * chunk_div), 1..64
    int wg_dmax = 0;             // workgroup-tier out-degree limit (0: as LDS allows); larger roots go to scratch
    int local_bits = 128;        // widest local graph candidate sets are compacted into (64 or 128 nodes)
    int wg_waves = 0;            // waves per workgroup-tier block (0: chosen per launch)
};
const kc_tuning_t &kc_tuning_now();

// Scheduler (kc_sched.hip)
#define KC_WG_CLASSES 16
#define KC_RES_WORDS 1072  // per-count result block: total, overflow flag, u32 queue counters, total slots
#define KC_RES_SLOTS 1040  // first of the 32 partial-total words (summed into word 0 at the end)
#define KC_MLP_IN 8
#define KC_MLP_H 32
static_assert(KC_MLP_PARAMS == KC_MLP_IN * KC_MLP_H + KC_MLP_H + KC_MLP_H * KC_MLP_H + KC_MLP_H + KC_MLP_H + 1,
              "KC_MLP_PARAMS of kc.h");
struct kc_queue {
    kc_tmp buf;                // storage when the queue is built per call
    kc_tmp items_buf;
    const uint64_t *wg_items = nullptr;  // workgroup tier as split items (see KC_ITEM_LEVEL2 below)
    uint32_t wg_item_count = 0;
    bool wg_l2 = false;                  // the items include two-level items
    // the tier's roots of out-degree up to wg_dmax2 as items of their own (after the
    // larger roots' wg_items, which then cover only those above wg_dmax2)
    const uint64_t *wg_items2 = nullptr;
    uint32_t wg_item_count2 = 0;
    bool wg_l2b = false;
    uint32_t wg_dmax2 = 0;
    const uint32_t *ptr[3];    // root ranks of each tier (wave, workgroup, scratch), heaviest first
    uint32_t count[3];         // roots per tier
    uint32_t max_d[3];         // largest out-degree in each tier
    // workgroup tier sorted by out-degree (descending): runs of one class
    // (2^j, 2^(j+1)] of out-degrees, each launched with an arena sized for it
    uint32_t wg_ncls = 0;
    uint32_t wg_cls_off[KC_WG_CLASSES], wg_cls_cnt[KC_WG_CLASSES], wg_cls_dmax[KC_WG_CLASSES];
};
// no_alloc: degree policy only, from the handle's degree queue and work items as they
// already are (KC_ESTATE when the degree queue is not built); nothing is allocated,
// and heavy roots stay whole when the handle holds no work items for this tier.
// Packed upper-triangular bitmap of G+(u) with d nodes and W = ceil(d / 64) words per
// row: row i holds words floor((i+1)/64) .. W-1 and starts at word
// i*W - sum_{t=1}^{i} floor(t/64) of the root's bitmap.
__host__ __device__ inline uint64_t kc_tri_rowoff(uint64_t i, uint64_t W) {
    const uint64_t q = i >> 6, r = i & 63;
    return i * W - (64 * (q * (q - (q ? 1 : 0)) / 2) + q * (r + 1));
}

// Workgroup-tier work items (64 bits): the root's rank in the high half, and in the
// low half either
//   t << 22 | part << 16 | parts (1..64) [| KC_ITEM_SKIP_WIDE]: the root's first-level
//       nodes part, part + parts, ...; with the flag, those whose candidate set held
//       more than t (> KC_ITEM_WIDE) nodes when staged are left to two-level items;
//   v << 16 | KC_ITEM_LEVEL2 | part2 << 7 | parts2 (2..127): first-level node v only,
//       the cliques whose second-level node index is part2 mod parts2.
// A rank of 0xFFFFFFFF is padding.
constexpr uint32_t KC_ITEM_LEVEL2 = 1u << 15;
constexpr uint32_t KC_ITEM_SKIP_WIDE = 1u << 14;
constexpr uint32_t KC_ITEM_WIDE = 128;
kc_status kc_build_queue(const kc_graph *g, int k, int policy, uint32_t d_lds_max, kc_queue &q,
                         bool no_alloc = false);
size_t kc_scratch_slice_words(uint32_t dmax, int k);
// Inference and queue keys of the learned policy for the candidate roots dq[0, C)
// (kc_mlp.hip; key layout in kc_learned_prio below).
kc_status kc_learned_keys(const kc_graph *g, int k, uint32_t C, uint32_t wd, uint32_t dcap, float promote,
                          uint64_t *keys, uint32_t *stats, hipStream_t s);
// 24-bit queue priority of a predicted log-work (2^-18 steps, larger work first) and back
__host__ __device__ inline uint32_t kc_learned_prio(float logwork) {
    float v = logwork * 262144.0f;
    v = v < 0.f ? 0.f : (v > 16777215.f ? 16777215.f : v);
    return 0xFFFFFFu - (uint32_t)v;
}
__host__ __device__ inline double kc_learned_logwork(uint32_t prio) { return (double)(0xFFFFFFu - prio) / 262144.0; }

// ----------------------------------------------------------------------------
// Wave64 helpers
#ifdef __HIP_DEVICE_COMPILE__
#define KC_DEV __device__ __forceinline__
#else
#define KC_DEV __device__ inline
#endif

KC_DEV uint32_t kc_lane() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
KC_DEV uint64_t kc_lanemask_lt() { return (1ull << kc_lane()) - 1ull; }

// LDS writes of a wave made visible to the wave's other lanes
KC_DEV void kc_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// position of the r-th set bit (r from 0) of w; w must have more than r bits set
KC_DEV uint32_t kc_select_bit(uint64_t w, uint32_t r) {
    uint32_t pos = 0;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const uint32_t c = (uint32_t)__popcll(w & ((1ull << s) - 1ull));
        if (r >= c) {
            r -= c;
            w >>= s;
            pos += s;
        }
    }
    return pos;
}

// largest i in [0, d) with seg[i] <= e  (seg[0] = 0 <= e)
KC_DEV uint32_t kc_seg_find(const uint32_t *seg, uint32_t d, uint32_t e) {
    uint32_t lo = 0, hi = d;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (seg[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// SplitMix64 finaliser (Steele, Lea & Flood 2014)
__host__ __device__ inline uint64_t kc_mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint32_t kc_colour(uint64_t h, uint32_t c) {
    return (uint32_t)(((h >> 32) * (uint64_t)c) >> 32);
}

KC_DEV uint64_t kc_wave_sum_u64(uint64_t v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
KC_DEV uint32_t kc_wave_sum_u32(uint32_t v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
KC_DEV uint32_t kc_wave_max_u32(uint32_t v) {
    for (int off = 32; off >= 1; off >>= 1) {
        uint32_t o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}
// Exact wave-wide sum of 64-bit values; sets *ovf if the sum needs more than 64 bits.
KC_DEV uint64_t kc_wave_sum_checked(uint64_t v, int *ovf) {
    uint64_t lo = kc_wave_sum_u64(v & 0xffffffffull);
    uint64_t hi = kc_wave_sum_u64(v >> 32);
    if (hi >> 32) *ovf = 1;
    uint64_t t = hi << 32, r = t + lo;
    if (r < t) *ovf = 1;
    return r;
}
// inclusive prefix sum across the wave
KC_DEV uint32_t kc_wave_incl_u32(uint32_t v) {
    const uint32_t lane = kc_lane();
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v += o;
    }
    return v;
}
