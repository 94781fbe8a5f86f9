// Work queues for the counting kernels.
//
// The paper observes that round-3 reducers are heavily skewed ("curse of the
// last reducer", Section 5) and suggests giving heavy high-neighbourhoods more
// resources (Section 7).  Here every root u with |Gamma+(u)| >= k-1 (smaller
// roots hold no (k-1)-clique: the Reduce-1 filter of Algorithm 1) is placed in
// a tier and the queue of each tier is ordered heaviest first:
//   degree policy    tier by out-degree, order by out-degree, whole roots.  The
//                    order does not depend on k, so the queue is sorted once per
//                    graph; for a given k the tiers are prefixes read off an
//                    out-degree histogram (the one-wave part stops at k-1).
//   edges policy     the degree queue, but from k = 5 the workgroup tier becomes
//                    items ordered and split by an estimate from the edges of
//                    G+(u) (known once staged; by out-degree without the cache).
//   learned policy   from k = 5 the workgroup tier's items ordered and split by
//                    an MLP's predicted work, and one-wave roots whose predicted
//                    work is large promoted to the workgroup tier; built once per
//                    clique size and weights.  Below k = 5 no one-wave root can
//                    reach the promotion threshold and the queue is the degree
//                    queue.
#include <string.h>

#include "kc_internal.h"

namespace {

constexpr int T = 256;
inline unsigned grid_for(size_t n) { return (unsigned)((n + T - 1) / T); }
constexpr uint32_t HIST_LDS = 1024;  // out-degrees below this are binned in LDS first

// key = part (wide/narrow) | 24-bit out-degree complement | rank
__global__ void k_degree_keys(const uint64_t *optr, uint32_t n, uint32_t wd, uint32_t dmax, int db,
                              uint64_t *keys, uint32_t *flag, uint32_t *hist) {
    __shared__ uint32_t s_h[HIST_LDS];
    for (uint32_t i = threadIdx.x; i < HIST_LDS; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) {
        // sort key above the rank: wave-tier bit, then dmax - d (larger out-degree first)
        const uint32_t d = (uint32_t)(optr[u + 1] - optr[u]);
        keys[u] = ((uint64_t)(d <= wd ? 1u : 0u) << (32 + db)) | ((uint64_t)(dmax - d) << 32) | (uint64_t)u;
        flag[u] = d >= 2 ? 1u : 0u;
        if (d < HIST_LDS) atomicAdd(&s_h[d], 1u);
        else atomicAdd(&hist[d], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < HIST_LDS; i += blockDim.x)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

__global__ void k_compact_keys(const uint64_t *keys, const uint32_t *flag, const uint32_t *pos, uint32_t n,
                               uint64_t *out) {
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n && flag[u]) out[pos[u]] = keys[u];
}

__global__ void k_queue_from_keys(const uint64_t *keys, uint32_t cnt, uint32_t *queue) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) queue[i] = (uint32_t)keys[i];
}

__global__ void k_split_emit(const uint32_t *q, uint32_t cnt, const uint32_t *parts, const uint32_t *off,
                             uint64_t *items) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const uint32_t np = parts[i];
    for (uint32_t pt = 0; pt < np; ++pt)
        items[off[i] + pt] = ((uint64_t)q[i] << 32) | ((uint64_t)pt << 16) | (uint64_t)np;
}

// Split of the workgroup tier (degree policy): a root of out-degree d above dsplit
// is cut into parts(d) = min(ceil(d / 2^sh), 64) items.
__host__ __device__ inline uint32_t degree_parts(uint64_t d, uint32_t dsplit, uint32_t sh) {
    if (d <= dsplit) return 1u;
    const uint64_t np = (d + (1ull << sh) - 1) >> sh;
    return np > 64 ? 64u : (uint32_t)np;
}

__global__ void k_degree_parts(const uint32_t *q, uint32_t cnt, const uint64_t *optr, uint32_t dsplit, uint32_t sh,
                               uint32_t *parts) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const uint32_t u = q[i];
    parts[i] = degree_parts(optr[u + 1] - optr[u], dsplit, sh);
}

// Work items of the workgroup tier, three grid passes and no host round trip:
//   1. the sum of the roots' estimated work;
//   2. items per root, ceil(est / target) with target the smaller of four times
//      the mean and 1/1024 of the total (at least 1), at most min(64, out-degree);
//      items per 8-bit estimate bucket;
//   3. items written bucket by bucket, heaviest bucket first (a counting sort:
//      longest-processing-time order at bucket resolution), the list padded to
//      its bound with skipped items.
// Items: sum of parts <= cnt + total / target <= cnt + max(cnt / 4, 1024).
// The estimate is either the edge estimate below (KC_SCHED_EDGES, from the edges
// of G+(u) kept when staging) or the MLP's predicted work (KC_SCHED_LEARNED):
// the same machinery, only the per-root estimate differs.
struct WqAux {
    double sum;
    uint32_t bcnt[256];  // items per bucket
    uint32_t bcur[256];  // items placed per bucket
};

__global__ void k_wq_clear(WqAux *a) {
    const uint32_t t = threadIdx.x;
    if (t == 0) a->sum = 0.0;
    for (uint32_t i = t; i < 256; i += blockDim.x) {
        a->bcnt[i] = 0;
        a->bcur[i] = 0;
    }
}

// Estimated work of a root from the edges c and nodes d of G+(u): c^1.5 / d^2
// (time grows with the size and the density of G+(u)), in 1/64 units, saturated.
__device__ __forceinline__ uint32_t root_est(uint32_t c, uint64_t d) {
    const double dd = d ? (double)d : 1.0;
    const double e = 64.0 * (double)c * sqrt((double)c) / (dd * dd);
    return e >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)e;
}

// Root i of a tier with its edge estimate (queue of ranks, staged edge counts)
struct EstEdges {
    const uint32_t *q;
    const uint32_t *wedges;
    const uint64_t *optr;
    const uint64_t *wbits, *woff;  // the staged bitmaps (two-level items), or null
    __device__ uint32_t rank(size_t i) const { return q[i]; }
    __device__ uint64_t outdeg(size_t i) const { return optr[q[i] + 1] - optr[q[i]]; }
    __device__ uint32_t est(size_t i) const { return root_est(wedges[q[i]], outdeg(i)); }
};

// Learned queue keys: tier (2 bits) | 24-bit priority of the predicted log-work
// (kc_learned_prio) | rank; the estimate is the predicted work, in 1/64 units.
struct EstLearned {
    const uint64_t *keys;
    const uint64_t *optr;
    const uint64_t *wbits, *woff;  // the staged bitmaps (two-level items), or null
    __device__ uint32_t rank(size_t i) const { return (uint32_t)keys[i]; }
    __device__ uint64_t outdeg(size_t i) const { return optr[rank(i) + 1] - optr[rank(i)]; }
    __device__ uint32_t est(size_t i) const {
        const uint32_t prio = (uint32_t)(keys[i] >> 32) & 0xFFFFFFu;
        const double e = 64.0 * expm1(kc_learned_logwork(prio));
        return e >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)e;
    }
};

template <class Est>
__global__ void k_est_sum(Est E, uint32_t cnt, WqAux *a) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t c = i < cnt ? E.est(i) : 0u;
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63u) == 0 && c) atomicAdd(&a->sum, (double)c);
}

// 8-bit bucket of an estimate, larger first: 255 - (8 * floor(log2 c) + the next
// three bits of c).
__device__ __forceinline__ uint32_t est_bucket(uint32_t c) {
    if (c == 0) return 255u;
    const uint32_t e = 31u - (uint32_t)__builtin_clz(c);
    const uint32_t m = e >= 3 ? (c >> (e - 3)) & 7u : (c << (3 - e)) & 7u;
    const uint32_t key = 8u * e + m;
    return 255u - (key > 255u ? 255u : key);
}

template <class Est>
__global__ void k_root_parts(Est E, uint32_t cnt, WqAux *a, uint32_t *parts) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const double tot = a->sum;
    double target = 4.0 * tot / (double)cnt;
    if (tot / 1024.0 < target) target = tot / 1024.0;
    if (target < 1.0) target = 1.0;
    const uint64_t d = E.outdeg(i);
    const uint32_t c = E.est(i);
    double np = ceil((double)c / target);
    const double cap = d < 64 ? (double)(d ? d : 1) : 64.0;
    np = np < 1.0 ? 1.0 : (np > cap ? cap : np);
    parts[i] = (uint32_t)np;
    atomicAdd(&a->bcnt[est_bucket(c)], (uint32_t)np);
}

constexpr uint32_t WQ_SKIP = 0xFFFFFFFFu;

// Two-level items (Section 7, the further split of the heaviest sub-problems): in a
// root cut into several items, every first-level node v whose candidate set holds more
// than KC_ITEM_WIDE nodes gets parts2 items of its own, ceil(est_v / target) with est_v
// the root's estimate times pc_v^2 / sum over the root's nodes of pc^2 (pc = candidate
// set size); the root's first-level items then skip those nodes.  One block per root:
// n2[i] = two-level items of root i (0 for roots that are not split).
constexpr int L2T = 256;
// Per root: the split threshold t (nodes whose candidate set holds more than t nodes
// get two-level items: est_v = est * pc^2 / S2 >= 2 target, i.e. pc >= sqrt(2 target
// S2 / est); at least KC_ITEM_WIDE + 1, the wide search's nodes; 1023 = none) and the
// items of one such node, ceil(est_v / target) in 2..127.  force (KC_LEVEL2=2) splits
// every wide node in two at least.
__device__ __forceinline__ uint32_t level2_threshold(double est, double S2, double target, bool force) {
    if (force) return KC_ITEM_WIDE;
    if (est <= 0.0) return 1023u;
    const double t = ceil(sqrt(2.0 * target * S2 / est));
    if (t >= 1023.0) return 1023u;
    return t <= (double)KC_ITEM_WIDE ? KC_ITEM_WIDE : (uint32_t)t;
}
__device__ __forceinline__ uint32_t level2_parts(double est, double S2, double target, uint32_t pc, bool force) {
    double np = S2 > 0.0 ? ceil(est * (double)pc * (double)pc / S2 / target) : 2.0;
    np = np < 2.0 ? 2.0 : (np > 127.0 ? 127.0 : np);
    (void)force;
    return (uint32_t)np;
}

template <class Est>
__global__ void __launch_bounds__(L2T) k_level2_count(Est E, const uint32_t *parts, uint32_t cnt, const WqAux *a,
                                                     bool force, uint32_t *n2, uint32_t *thr) {
    __shared__ double s_sum[L2T / 64];
    __shared__ uint32_t s_cnt[L2T / 64];
    const uint32_t i = blockIdx.x;
    if (i >= cnt) return;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    // a wide node needs more than KC_ITEM_WIDE later nodes, so the root more than
    // KC_ITEM_WIDE + 1 nodes: such roots keep a packed bitmap (above the one-wave limit)
    const uint32_t d = (uint32_t)E.outdeg(i), W = (d + 63) / 64;
    if (parts[i] < 2 || !E.wbits || d <= KC_ITEM_WIDE + 1) {
        if (tid == 0) {
            n2[i] = 0;
            thr[i] = 1023u;
        }
        return;
    }
    const uint32_t u = E.rank(i);
    const uint64_t *bm = E.wbits + E.woff[u];
    auto pc_of = [&](uint32_t j) {
        const uint64_t *rj = bm + kc_tri_rowoff(j, W) - ((j + 1) >> 6);
        uint32_t c = 0;
        for (uint32_t l = (j + 1) >> 6; l < W; ++l) c += (uint32_t)__popcll(rj[l]);
        return c;
    };
    double sq = 0.0;
    for (uint32_t j = tid; j < d; j += L2T) {
        const double c = (double)pc_of(j);
        sq += c * c;
    }
    for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if (lane == 0) s_sum[wave] = sq;
    __syncthreads();
    double S2 = 0.0;
    for (int w = 0; w < L2T / 64; ++w) S2 += s_sum[w];
    const double tot = a->sum;
    double target = 4.0 * tot / (double)cnt;
    if (tot / 1024.0 < target) target = tot / 1024.0;
    if (target < 1.0) target = 1.0;
    const double est = (double)E.est(i);
    const uint32_t t = level2_threshold(est, S2, target, force);
    uint32_t items = 0;
    for (uint32_t j = tid; j < d; j += L2T) {
        const uint32_t c = pc_of(j);
        if (c > t) items += level2_parts(est, S2, target, c, force);
    }
    items = kc_wave_sum_u32(items);
    if (lane == 0) s_cnt[wave] = items;
    __syncthreads();
    if (tid == 0) {
        uint32_t sum = 0;
        for (int w = 0; w < L2T / 64; ++w) sum += s_cnt[w];
        n2[i] = sum;
        thr[i] = sum ? t : 1023u;
    }
}

// The two-level items of root i at items[off2[i] ..), in node order.
template <class Est>
__global__ void __launch_bounds__(L2T) k_level2_emit(Est E, const uint32_t *parts, uint32_t cnt, const WqAux *a,
                                                    bool force, const uint32_t *n2, const uint32_t *off2,
                                                    const uint32_t *thr, uint64_t *items) {
    __shared__ double s_sum[L2T / 64];
    __shared__ uint32_t s_pos;
    const uint32_t i = blockIdx.x;
    if (i >= cnt || n2[i] == 0) return;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t u = E.rank(i);
    const uint32_t d = (uint32_t)E.outdeg(i), W = (d + 63) / 64;
    const uint64_t *bm = E.wbits + E.woff[u];
    auto pc_of = [&](uint32_t j) {
        const uint64_t *rj = bm + kc_tri_rowoff(j, W) - ((j + 1) >> 6);
        uint32_t c = 0;
        for (uint32_t l = (j + 1) >> 6; l < W; ++l) c += (uint32_t)__popcll(rj[l]);
        return c;
    };
    double sq = 0.0;
    for (uint32_t j = tid; j < d; j += L2T) {
        const double c = (double)pc_of(j);
        sq += c * c;
    }
    for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if (lane == 0) s_sum[wave] = sq;
    if (tid == 0) s_pos = 0;
    __syncthreads();
    double S2 = 0.0;
    for (int w = 0; w < L2T / 64; ++w) S2 += s_sum[w];
    const double tot = a->sum;
    double target = 4.0 * tot / (double)cnt;
    if (tot / 1024.0 < target) target = tot / 1024.0;
    if (target < 1.0) target = 1.0;
    const double est = (double)E.est(i);
    const uint32_t t = thr[i];
    for (uint32_t j = tid; j < d; j += L2T) {
        const uint32_t c = pc_of(j);
        if (c <= t) continue;
        const uint32_t m = level2_parts(est, S2, target, c, force);
        const uint32_t at = off2[i] + atomicAdd(&s_pos, m);
        for (uint32_t p2 = 0; p2 < m; ++p2)
            items[at + p2] = ((uint64_t)u << 32) | ((uint64_t)j << 16) | KC_ITEM_LEVEL2 | ((uint64_t)p2 << 7) | m;
    }
}

template <class Est>
__global__ void k_emit_items(Est E, const uint32_t *parts, const uint32_t *n2, const uint32_t *thr, uint32_t cnt,
                             WqAux *a, uint32_t bound, uint64_t *items) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t s_total;
    const uint32_t tid = threadIdx.x;
    if (tid < 64) {  // exclusive scan of the 256 bucket counts, four per lane
        const uint32_t h0 = a->bcnt[4 * tid], h1 = a->bcnt[4 * tid + 1], h2 = a->bcnt[4 * tid + 2],
                       h3 = a->bcnt[4 * tid + 3];
        const uint32_t t4 = h0 + h1 + h2 + h3;
        const uint32_t incl = kc_wave_incl_u32(t4);
        const uint32_t b0 = incl - t4;
        base[4 * tid] = b0;
        base[4 * tid + 1] = b0 + h0;
        base[4 * tid + 2] = b0 + h0 + h1;
        base[4 * tid + 3] = b0 + h0 + h1 + h2;
        if (tid == 63) s_total = incl;
    }
    __syncthreads();
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + tid; i < cnt; i += stride) {
        const uint32_t u = E.rank(i), b = est_bucket(E.est(i)), np = parts[i];
        const uint32_t off = base[b] + atomicAdd(&a->bcur[b], np);
        const uint64_t flag = n2 && n2[i] ? (KC_ITEM_SKIP_WIDE | ((uint64_t)thr[i] << 22)) : 0u;
        for (uint32_t pt = 0; pt < np; ++pt)
            if (off + pt < bound) items[off + pt] = ((uint64_t)u << 32) | ((uint64_t)pt << 16) | flag | (uint64_t)np;
    }
    for (size_t x = s_total + (size_t)blockIdx.x * blockDim.x + tid; x < bound; x += stride)
        items[x] = (uint64_t)WQ_SKIP << 32;
}

// Bound of the item count; the list is padded to it.
inline uint32_t work_items_bound(uint32_t cnt) {
    const uint32_t extra = (cnt + 3) / 4 > 1024u ? (cnt + 3) / 4 : 1024u;
    return cnt + extra + 1;
}

// Items of cnt roots into a new device list (owned by the caller, *count entries):
// the two-level items of the heaviest nodes first (when the staged bitmaps are given
// and KC_LEVEL2 is not 0), then the roots' first-level items in estimate order,
// padded to their bound.
template <class Est>
kc_status build_items(const Est &E, uint32_t cnt, hipStream_t s, uint64_t **items, uint32_t *count, bool *l2out) {
    const uint32_t bound = work_items_bound(cnt);
    kc_tmp aux, parts, n2, off2, tot2;
    KC_TRY(kc_tmp_alloc(aux, sizeof(WqAux), s));
    KC_TRY(kc_tmp_alloc(parts, (size_t)cnt * 4, s));
    WqAux *a = aux.as<WqAux>();
    hipLaunchKernelGGL(k_wq_clear, dim3(1), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_est_sum<Est>, dim3(grid_for(cnt)), dim3(T), 0, s, E, cnt, a);
    hipLaunchKernelGGL(k_root_parts<Est>, dim3(grid_for(cnt)), dim3(T), 0, s, E, cnt, a, parts.as<uint32_t>());
    KC_HIP(hipGetLastError());
    uint32_t N2 = 0;
    // KC_LEVEL2: 0 no two-level items, 2 every wide node of a split root split (tests)
    const char *l2 = getenv("KC_LEVEL2");
    const bool level2 = E.wbits && !(l2 && l2[0] == '0') && cnt;
    const bool force = l2 && l2[0] == '2';
    kc_tmp thr;
    if (level2) {
        KC_TRY(kc_tmp_alloc(n2, (size_t)cnt * 4, s));
        KC_TRY(kc_tmp_alloc(thr, (size_t)cnt * 4, s));
        KC_TRY(kc_tmp_alloc(off2, (size_t)cnt * 4, s));
        KC_TRY(kc_tmp_alloc(tot2, 4, s));
        hipLaunchKernelGGL(k_level2_count<Est>, dim3(cnt), dim3(L2T), 0, s, E, (const uint32_t *)parts.as<uint32_t>(),
                           cnt, (const WqAux *)a, force, n2.as<uint32_t>(), thr.as<uint32_t>());
        KC_HIP(hipGetLastError());
        KC_TRY(kc_scan_excl_u32(n2.as<uint32_t>(), off2.as<uint32_t>(), cnt, tot2.as<uint32_t>(), s));
        uint32_t *h = (uint32_t *)kc_pinned_scratch();
        KC_HIP(hipMemcpyAsync(h, tot2.p, 4, hipMemcpyDeviceToHost, s));
        KC_TRY(kc_sync(s));
        N2 = h[0];
    }
    KC_TRY(kc_dev_alloc((void **)items, ((size_t)bound + N2) * 8, s));
    if (N2)
        hipLaunchKernelGGL(k_level2_emit<Est>, dim3(cnt), dim3(L2T), 0, s, E, (const uint32_t *)parts.as<uint32_t>(),
                           cnt, (const WqAux *)a, force, (const uint32_t *)n2.as<uint32_t>(),
                           (const uint32_t *)off2.as<uint32_t>(), (const uint32_t *)thr.as<uint32_t>(), *items);
    hipLaunchKernelGGL(k_emit_items<Est>, dim3(grid_for(bound)), dim3(T), 0, s, E,
                       (const uint32_t *)parts.as<uint32_t>(), level2 ? (const uint32_t *)n2.as<uint32_t>() : nullptr,
                       level2 ? (const uint32_t *)thr.as<uint32_t>() : nullptr, cnt, a, bound, *items + N2);
    KC_HIP(hipGetLastError());
    *count = bound + N2;
    *l2out = N2 > 0;
    return KC_OK;
}

// The workgroup tier's items for its cnt roots from queue position first (out-degree
// descending), split at out-degree dsplit when that leaves roots on both sides: the
// nbig roots above it in g->wq, the rest in g->wq2.
kc_status build_work_items(kc_graph *g, uint32_t first, uint32_t cnt, uint32_t dsplit, uint32_t nbig) {
    hipStream_t s = g->stream;
    kc_cache_free(g->wq, s);
    kc_cache_free(g->wq2, s);
    g->wq = g->wq2 = nullptr;
    g->wq_count = g->wq2_count = 0;
    g->wq_l2 = g->wq2_l2 = false;
    g->wq_ready = 0;
    if (nbig == 0 || nbig >= cnt) dsplit = 0;
    const uint32_t n1 = dsplit ? nbig : cnt;
    EstEdges E{g->dq + first, g->wedges, g->optr, g->wbits, g->woff};
    uint32_t bound = 0;
    KC_TRY(build_items(E, n1, s, &g->wq, &bound, &g->wq_l2));
    g->wq_count = bound;
    if (dsplit) {
        EstEdges E2{g->dq + first + nbig, g->wedges, g->optr, g->wbits, g->woff};
        KC_TRY(build_items(E2, cnt - nbig, s, &g->wq2, &bound, &g->wq2_l2));
        g->wq2_count = bound;
    }
    g->wq_dsplit = dsplit;
    g->wq_first = first;
    g->wq_roots = cnt;
    g->wq_ready = 1;
    return KC_OK;
}

kc_status build_degree_cache(kc_graph *g, uint32_t wd) {
    hipStream_t s = g->stream;
    if (g->dq) {
        kc_cache_free(g->dq, s);
        g->dq = nullptr;
    }
    delete[] g->dq_hist;
    g->dq_hist = nullptr;
    g->dq_ready = 0;
    const uint32_t n = g->n;
    const uint32_t hn = g->max_outdeg + 1;
    kc_tmp keys, keys2, tmp, flag, pos, hist, total;
    KC_TRY(kc_tmp_alloc(keys, (size_t)n * 8, s));
    KC_TRY(kc_tmp_alloc(flag, (size_t)n * 4, s));
    KC_TRY(kc_tmp_alloc(pos, (size_t)n * 4, s));
    const uint32_t hcap = hn > HIST_LDS ? hn : HIST_LDS;
    KC_TRY(kc_tmp_alloc(hist, (size_t)hcap * 4, s));
    KC_TRY(kc_tmp_alloc(total, 8, s));
    KC_HIP(hipMemsetAsync(hist.p, 0, (size_t)hcap * 4, s));
    int db = 1;  // bits of dmax - d
    while (db < 31 && ((uint64_t)1 << db) <= (uint64_t)g->max_outdeg) ++db;
    hipLaunchKernelGGL(k_degree_keys, dim3(grid_for(n)), dim3(T), 0, s, (const uint64_t *)g->optr, n, wd,
                       g->max_outdeg, db, keys.as<uint64_t>(), flag.as<uint32_t>(), hist.as<uint32_t>());
    KC_HIP(hipGetLastError());
    KC_TRY(kc_scan_excl_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), n, total.as<uint32_t>(), s));
    uint32_t *h = (uint32_t *)kc_pinned_buffer(((size_t)hn + 1) * 4);
    if (!h) return kc_fail(KC_ENOMEM, "pinned host histogram");
    KC_HIP(hipMemcpyAsync(h, hist.p, (size_t)hn * 4, hipMemcpyDeviceToHost, s));
    KC_HIP(hipMemcpyAsync(h + hn, total.p, 4, hipMemcpyDeviceToHost, s));
    KC_TRY(kc_sync(s));
    const uint32_t active = h[hn];
    g->dq_hist = new (std::nothrow) uint64_t[hn];
    if (!g->dq_hist) return kc_fail(KC_ENOMEM, "host histogram");
    uint32_t wide = 0;
    for (uint32_t d = 0; d < hn; ++d) {
        g->dq_hist[d] = h[d];
        if (d > wd) wide += h[d];
    }
    g->dq_wide = wide;
    g->dq_narrow = active - wide;
    KC_TRY(kc_dev_alloc((void **)&g->dq, (size_t)(active ? active : 1) * 4, s));
    if (active) {
        KC_TRY(kc_tmp_alloc(keys2, (size_t)active * 8, s));
        KC_TRY(kc_tmp_alloc(tmp, (size_t)active * 8, s));
        hipLaunchKernelGGL(k_compact_keys, dim3(grid_for(n)), dim3(T), 0, s, (const uint64_t *)keys.as<uint64_t>(),
                           (const uint32_t *)flag.as<uint32_t>(), (const uint32_t *)pos.as<uint32_t>(), n,
                           keys2.as<uint64_t>());
        KC_HIP(hipGetLastError());
        KC_TRY(kc_radix_sort_u64(keys2.as<uint64_t>(), tmp.as<uint64_t>(), active, 32, 33 + db, s));
        hipLaunchKernelGGL(k_queue_from_keys, dim3(grid_for(active)), dim3(T), 0, s,
                           (const uint64_t *)keys2.as<uint64_t>(), active, g->dq);
        KC_HIP(hipGetLastError());
    }
    g->dq_wd = (int)wd;
    g->dq_ready = 1;
    return KC_OK;
}

}  // namespace

// Smallest out-degree d in [lo, hi] whose unpruned work bound, the number of l-cliques
// of a complete G+(u) for l = 1..k-2, reaches e^promote; hi + 1 if none does.
static uint32_t promote_outdeg(int k, float promote, uint32_t lo, uint32_t hi) {
    for (uint32_t d = lo; d <= hi; ++d) {
        double c = 1.0, w = 0.0;
        for (int l = 1; l <= k - 2; ++l) {
            c = c * (double)(d - l + 1) / (double)l;
            w += c;
        }
        if (w > 0.0 && log(w) >= (double)promote) return d;
    }
    return hi + 1;
}

// Out-degree at which the workgroup tier's roots split into two item lists, each
// launched with an arena of its own size (0: one list).  The roots above half the
// tier's largest out-degree get items of their own, launched with an arena of that
// size on a second stream beside the others' items with an arena of half the size
// (about a quarter of the bytes: more blocks per CU).  Measured split points: R-MAT 22
// k = 5 (out-degrees to 1031): one list 1.28 s, 384 / 512 / 640 / 768: 641 / 609 / 641
// / 815 ms; planted 4M k = 5..8 (to 519): one list 16.9 / 42.7 / 138 / 266 ms, 256:
// 16.1 / 40.9 / 136 / 259 ms, 160 or 400: between.  KC_WG_DSPLIT (test hook) sets it.
static uint32_t choose_dsplit(const kc_graph *g, int k, uint32_t wd, uint32_t top) {
    const char *ds = getenv("KC_WG_DSPLIT");
    uint32_t dsplit = 0;
    if (ds)
        dsplit = (uint32_t)atoi(ds);
    else if (top > 2u * wd && kc_wg_blocks_per_cu(g->device, k, top / 2) > kc_wg_blocks_per_cu(g->device, k, top))
        dsplit = top / 2;
    return dsplit > wd && dsplit < top ? dsplit : 0u;
}

// stable partition of n learned keys: those of roots above out-degree dsplit first
__global__ void k_part_flags(const uint64_t *keys, uint32_t n, const uint64_t *optr, uint32_t dsplit,
                             uint32_t *flag) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t r = (uint32_t)keys[i];
    flag[i] = optr[r + 1] - optr[r] > dsplit ? 1u : 0u;
}
__global__ void k_part_scatter(const uint64_t *keys, uint32_t n, const uint32_t *flag, const uint32_t *pos,
                               const uint32_t *nbig, uint64_t *out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[flag[i] ? pos[i] : *nbig + (uint32_t)i - pos[i]] = keys[i];
}

// Learned queue of clique size k (cached on the handle): candidates are the roots
// above the one-wave limit and the one-wave roots whose work bound reaches the
// promotion threshold, a prefix of the degree queue (sorted by out-degree).
static kc_status build_learned(kc_graph *g, int k, uint32_t wd, uint32_t dcap, kc_graph::LearnedQueue &L) {
    hipStream_t s = g->stream;
    const uint64_t *hist = g->dq_hist;
    const uint32_t dmax = g->max_outdeg;
    const char *pe = getenv("KC_PROMOTE_LOGWORK");
    const float promote = pe ? (float)atof(pe) : 14.0f;  // predicted work above ~1.2e6 intersections
    const uint32_t lo = (uint32_t)(k - 1) > 2u ? (uint32_t)(k - 1) : 2u;
    const uint32_t dmin = promote_outdeg(k, promote, lo, wd);
    uint32_t active = g->dq_wide, cand = g->dq_wide;
    for (uint32_t d = lo; d <= wd && d <= dmax; ++d) {
        active += (uint32_t)hist[d];
        if (d >= dmin) cand += (uint32_t)hist[d];
    }
    kc_cache_free(L.queue, s);
    kc_cache_free(L.items, s);
    kc_cache_free(L.items2, s);
    L = kc_graph::LearnedQueue();
    KC_TRY(kc_dev_alloc((void **)&L.queue, (size_t)(active ? active : 1) * 4, s));
    uint32_t h_stats[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    kc_tmp keys, tmp, stats;
    if (cand) {
        KC_TRY(kc_tmp_alloc(keys, (size_t)cand * 8, s));
        KC_TRY(kc_tmp_alloc(tmp, (size_t)cand * 8, s));
        KC_TRY(kc_tmp_alloc(stats, 8 * 4, s));
        KC_HIP(hipMemsetAsync(stats.p, 0, 8 * 4, s));
        KC_TRY(kc_learned_keys(g, k, cand, wd, dcap, promote, keys.as<uint64_t>(), stats.as<uint32_t>(), s));
        KC_TRY(kc_radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), cand, 32, 64, s));
        hipLaunchKernelGGL(k_queue_from_keys, dim3(grid_for(cand)), dim3(T), 0, s, (const uint64_t *)keys.as<uint64_t>(),
                           cand, L.queue);
        KC_HIP(hipGetLastError());
        uint32_t *h = (uint32_t *)kc_pinned_scratch();
        KC_HIP(hipMemcpyAsync(h, stats.p, 8 * 4, hipMemcpyDeviceToHost, s));
        KC_TRY(kc_sync(s));
        for (int i = 0; i < 8; ++i) h_stats[i] = h[i];
    }
    // the one-wave roots below the promotion bound keep their degree order after the candidates
    if (active > cand)
        KC_HIP(hipMemcpyAsync(L.queue + cand, g->dq + cand, (size_t)(active - cand) * 4, hipMemcpyDeviceToDevice, s));
    // kc_queue order: [0] one-wave, [1] workgroup, [2] scratch (the buffer holds them in reverse)
    L.count[2] = h_stats[0];
    L.count[1] = h_stats[1];
    L.count[0] = h_stats[2] + (active - cand);
    L.max_d[2] = h_stats[4];
    L.max_d[1] = h_stats[5];
    uint32_t wmax = h_stats[6];
    for (uint32_t d = lo; d < dmin && d <= wd && d <= dmax; ++d)
        if (hist[d]) wmax = d > wmax ? d : wmax;
    L.max_d[0] = wmax;
    if (k >= 5 && L.count[1]) {
        const bool bits = g->staged == 1 && g->stage_wd == (int)wd && g->wbits;
        const uint64_t *wk = keys.as<uint64_t>() + L.count[2];  // the workgroup tier, in priority order
        const uint32_t c1 = L.count[1];
        uint32_t dsplit = choose_dsplit(g, k, wd, L.max_d[1]);
        uint32_t nbig = 0;
        kc_tmp part, flag, pos, tot;
        if (dsplit) {
            // the tier's roots above dsplit first, each part in priority order
            KC_TRY(kc_tmp_alloc(part, (size_t)c1 * 8, s));
            KC_TRY(kc_tmp_alloc(flag, (size_t)c1 * 4, s));
            KC_TRY(kc_tmp_alloc(pos, (size_t)c1 * 4, s));
            KC_TRY(kc_tmp_alloc(tot, 4, s));
            hipLaunchKernelGGL(k_part_flags, dim3(grid_for(c1)), dim3(T), 0, s, wk, c1, (const uint64_t *)g->optr,
                               dsplit, flag.as<uint32_t>());
            KC_HIP(hipGetLastError());
            KC_TRY(kc_scan_excl_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), c1, tot.as<uint32_t>(), s));
            hipLaunchKernelGGL(k_part_scatter, dim3(grid_for(c1)), dim3(T), 0, s, wk, c1,
                               (const uint32_t *)flag.as<uint32_t>(), (const uint32_t *)pos.as<uint32_t>(),
                               (const uint32_t *)tot.as<uint32_t>(), part.as<uint64_t>());
            KC_HIP(hipGetLastError());
            uint32_t *h = (uint32_t *)kc_pinned_scratch();
            KC_HIP(hipMemcpyAsync(h, tot.p, 4, hipMemcpyDeviceToHost, s));
            KC_TRY(kc_sync(s));
            nbig = h[0];
            if (nbig == 0 || nbig >= c1) dsplit = 0;
        }
        const uint64_t *wbits = bits ? g->wbits : nullptr, *woff = bits ? g->woff : nullptr;
        if (dsplit) {
            EstLearned E{part.as<uint64_t>(), g->optr, wbits, woff};
            KC_TRY(build_items(E, nbig, s, &L.items, &L.item_count, &L.l2));
            EstLearned E2{part.as<uint64_t>() + nbig, g->optr, wbits, woff};
            KC_TRY(build_items(E2, c1 - nbig, s, &L.items2, &L.item_count2, &L.l2b));
            L.dsplit = dsplit;
        } else {
            EstLearned E{wk, g->optr, wbits, woff};
            KC_TRY(build_items(E, c1, s, &L.items, &L.item_count, &L.l2));
        }
    }
    L.wd = (int)wd;
    L.dcap = dcap;
    L.wserial = g->mlp_serial;
    L.ready = 1;
    return KC_OK;
}

kc_status kc_build_queue(const kc_graph *g, int k, int policy, uint32_t d_lds_max, kc_queue &q, bool no_alloc) {
    const uint32_t n = g->n;
    for (int t = 0; t < 3; ++t) {
        q.ptr[t] = nullptr;
        q.count[t] = q.max_d[t] = 0;
    }
    if (n == 0 || k < 3) return KC_OK;
    int wd = kc_tuning_now().wave_dmax;
    wd = wd < 1 ? 1 : (wd > 64 ? 64 : wd);
    if ((uint32_t)wd > d_lds_max) wd = (int)d_lds_max;
    kc_graph *gm = const_cast<kc_graph *>(g);
    if (no_alloc) policy = KC_SCHED_EDGES;
    if (policy == KC_SCHED_LEARNED && !g->mlp_loaded)
        return kc_fail(KC_ESTATE, "learned schedule requested but no MLP weights are loaded");
    if (!g->dq_ready || g->dq_wd != wd) {
        if (no_alloc) return kc_fail(KC_ESTATE, "the handle's degree queue is not built (count once with kc_count)");
        KC_TRY(build_degree_cache(gm, (uint32_t)wd));
    }
    if (policy == KC_SCHED_LEARNED && k >= 5) {
        kc_graph::LearnedQueue &L = gm->lq[k];
        if (!L.ready || L.wd != wd || L.dcap != d_lds_max || L.wserial != g->mlp_serial)
            KC_TRY(build_learned(gm, k, (uint32_t)wd, d_lds_max, L));
        q.ptr[2] = L.queue;
        q.ptr[1] = L.queue + L.count[2];
        q.ptr[0] = L.queue + L.count[2] + L.count[1];
        for (int t = 0; t < 3; ++t) {
            q.count[t] = L.count[t];
            q.max_d[t] = L.max_d[t];
        }
        q.wg_items = L.items;
        q.wg_item_count = L.items ? L.item_count : 0;
        q.wg_l2 = L.l2;
        if (L.dsplit) {
            q.wg_items2 = L.items2;
            q.wg_item_count2 = L.item_count2;
            q.wg_l2b = L.l2b;
            q.wg_dmax2 = L.dsplit;
        }
        q.wg_ncls = 0;
        return KC_OK;
    }
    {
        hipStream_t s = g->stream;
        const uint64_t *hist = g->dq_hist;
        const uint32_t dmax = g->max_outdeg;
        uint32_t scratch = 0, narrow = 0;
        for (uint32_t d = 0; d <= dmax; ++d) {
            if (!hist[d]) continue;
            if (d > d_lds_max) {
                scratch += (uint32_t)hist[d];
                q.max_d[2] = d;
            } else if (d > (uint32_t)wd) {
                q.max_d[1] = d;
            } else if (d >= (uint32_t)(k - 1)) {
                narrow += (uint32_t)hist[d];
                q.max_d[0] = d;
            }
        }
        q.ptr[2] = g->dq;
        q.count[2] = scratch;
        q.ptr[1] = g->dq + scratch;
        q.count[1] = g->dq_wide - scratch;
        q.ptr[0] = g->dq + g->dq_wide;
        q.count[0] = narrow;
        // out-degree classes of the workgroup tier, in queue order (largest first)
        q.wg_ncls = 0;
        uint32_t off = 0;
        int cur = -1;
        const uint32_t top = dmax < d_lds_max ? dmax : d_lds_max;
        for (uint32_t d = top; d > (uint32_t)wd; --d) {
            if (!hist[d]) continue;
            const int c = 31 - __builtin_clz(d - 1);
            if (c != cur) {
                if (q.wg_ncls == KC_WG_CLASSES) break;  // cannot happen for 32-bit out-degrees
                cur = c;
                q.wg_cls_off[q.wg_ncls] = off;
                q.wg_cls_cnt[q.wg_ncls] = 0;
                q.wg_cls_dmax[q.wg_ncls] = d;
                ++q.wg_ncls;
            }
            q.wg_cls_cnt[q.wg_ncls - 1] += (uint32_t)hist[d];
            off += (uint32_t)hist[d];
        }
        if (off != q.count[1]) q.wg_ncls = 0;  // not a plain degree order: one launch
        if (policy == KC_SCHED_DEGREE) return KC_OK;  // whole roots in out-degree order
        // From k = 5 on, the heaviest roots of the tier take most of its time, one
        // workgroup each: roots above twice the one-wave bound are split over
        // several items (Section 7, the (u, v) split), one per 32 first-level
        // nodes (64 at k = 5); item p takes the nodes p, p + parts, ...
        // With the staged cache, the tier is ordered by the edges of G+(u) instead
        // (a far better guess at a root's work than its out-degree; heaviest first,
        // longest-processing-time order) and split by that guess.
        const char *wo = getenv("KC_WORK_ORDER");
        if (k >= 5 && q.count[1] && g->staged == 1 && g->stage_wd == wd && g->wedges && !(wo && wo[0] == '0')) {
            const uint32_t first = (uint32_t)(q.ptr[1] - g->dq);
            uint32_t dsplit = choose_dsplit(g, k, (uint32_t)wd, top);
            uint32_t nbig = 0;
            if (dsplit)
                for (uint32_t d = dsplit + 1; d <= top; ++d) nbig += (uint32_t)hist[d];
            if (nbig == 0 || nbig >= q.count[1]) dsplit = 0;
            const bool have = g->wq_ready && g->wq_first == first && g->wq_roots == q.count[1] &&
                              g->wq_dsplit == dsplit;
            if (!have && no_alloc) return KC_OK;  // whole roots
            if (!have) KC_TRY(build_work_items(gm, first, q.count[1], dsplit, nbig));
            q.wg_items = g->wq;
            q.wg_item_count = g->wq_count;
            q.wg_l2 = g->wq_l2;
            if (g->wq_dsplit) {
                q.wg_items2 = g->wq2;
                q.wg_item_count2 = g->wq2_count;
                q.wg_l2b = g->wq2_l2;
                q.wg_dmax2 = g->wq_dsplit;
            }
            return KC_OK;
        }
        if (no_alloc) return KC_OK;
        // KC_DEGREE_SPLIT: 0 turns the split off, n > 0 sets 2^n nodes per item from k = 6 on
        const char *se = getenv("KC_DEGREE_SPLIT");
        const int sn = se ? atoi(se) : 6;
        if (k >= 5 && q.count[1] && sn > 0 && sn < 16) {
            const uint32_t dsplit = 2u * (uint32_t)wd, sh = (uint32_t)sn + (k >= 6 ? 0u : 1u);
            uint64_t nitems = 0;
            for (uint32_t d = (uint32_t)wd + 1; d <= top; ++d) nitems += hist[d] * degree_parts(d, dsplit, sh);
            const uint32_t c1 = q.count[1];
            if (nitems > c1 && nitems < (1ull << 32)) {
                kc_tmp parts, offs;
                KC_TRY(kc_tmp_alloc(parts, (size_t)c1 * 4, s));
                KC_TRY(kc_tmp_alloc(offs, (size_t)c1 * 4, s));
                KC_TRY(kc_tmp_alloc(q.items_buf, (size_t)nitems * 8, s));
                hipLaunchKernelGGL(k_degree_parts, dim3(grid_for(c1)), dim3(T), 0, s, q.ptr[1], c1,
                                   (const uint64_t *)g->optr, dsplit, sh, parts.as<uint32_t>());
                KC_HIP(hipGetLastError());
                KC_TRY(kc_scan_excl_u32(parts.as<uint32_t>(), offs.as<uint32_t>(), c1, nullptr, s));
                hipLaunchKernelGGL(k_split_emit, dim3(grid_for(c1)), dim3(T), 0, s, q.ptr[1], c1,
                                   (const uint32_t *)parts.as<uint32_t>(), (const uint32_t *)offs.as<uint32_t>(),
                                   q.items_buf.as<uint64_t>());
                KC_HIP(hipGetLastError());
                q.wg_items = q.items_buf.as<uint64_t>();
                q.wg_item_count = (uint32_t)nitems;
            }
        }
        return KC_OK;
    }
}
