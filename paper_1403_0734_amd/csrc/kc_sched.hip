// Work queues for the counting kernels.
//
// The paper observes that round-3 reducers are heavily skewed ("curse of the
// last reducer", Section 5) and suggests giving heavy high-neighbourhoods more
// resources (Section 7).  Here every root u with |Gamma+(u)| >= k-1 (smaller
// roots hold no (k-1)-clique: the Reduce-1 filter of Algorithm 1) is placed in
// a tier and the queue of each tier is ordered heaviest first:
//   degree policy   tier by out-degree, order by out-degree;
//   learned policy  order (and promotion of small but dense roots to the
//                   workgroup tier) by an MLP's predicted log-work.
#include "kc_internal.h"

namespace {

constexpr int T = 256;
inline unsigned grid_for(size_t n) { return (unsigned)((n + T - 1) / T); }

__device__ __forceinline__ void tier_stats(bool active, uint32_t tier, uint32_t d, uint32_t *cnt, uint32_t *mx) {
#pragma unroll
    for (uint32_t t = 0; t < 3; ++t) {
        const bool in = active && tier == t;
        const uint32_t c = (uint32_t)__popcll(__ballot(in));
        const uint32_t m = kc_wave_max_u32(in ? d : 0u);
        if ((threadIdx.x & 63) == 0 && c) {
            atomicAdd(&cnt[t], c);
            atomicMax(&mx[t], m);
        }
    }
}

// key = tier (2 bits) | 24-bit descending priority | rank
__global__ void k_bin(const uint64_t *optr, uint32_t n, int k, uint32_t dcap, const float *pred, float promote,
                      uint64_t *keys, uint32_t *flag, uint32_t *cnt, uint32_t *mx) {
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool active = false;
    uint32_t tier = 0, d = 0;
    if (u < n) {
        d = (uint32_t)(optr[u + 1] - optr[u]);
        active = d >= (uint32_t)(k - 1);
        tier = d <= 64 ? 0u : (d <= dcap ? 1u : 2u);
        uint32_t prio;
        if (pred) {
            const float w = pred[u];
            if (tier == 0 && w >= promote) tier = 1;
            float s = w * 262144.0f;  // log-work in 2^-18 steps
            s = s < 0.f ? 0.f : (s > 16777215.f ? 16777215.f : s);
            prio = 0xFFFFFFu - (uint32_t)s;
        } else {
            prio = 0xFFFFFFu - (d < 0xFFFFFFu ? d : 0xFFFFFFu);
        }
        keys[u] = ((uint64_t)tier << 62) | ((uint64_t)prio << 32) | (uint64_t)u;
        flag[u] = active ? 1u : 0u;
    }
    tier_stats(active, tier, d, cnt, mx);
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

}  // namespace

kc_status kc_predict_work(const kc_graph *g, float *d_pred, hipStream_t s);

kc_status kc_build_queue(const kc_graph *g, int k, int policy, uint32_t d_lds_max, kc_queue &q) {
    hipStream_t s = g->stream;
    const uint32_t n = g->n;
    for (int t = 0; t < 4; ++t) q.count[t] = q.offset[t] = q.max_d[t] = 0;
    if (n == 0 || k < 3) return KC_OK;

    kc_tmp keys, keys2, tmp, flag, pos, stats, pred;
    KC_TRY(kc_tmp_alloc(keys, (size_t)n * 8, s));
    KC_TRY(kc_tmp_alloc(flag, (size_t)n * 4, s));
    KC_TRY(kc_tmp_alloc(pos, (size_t)n * 4, s));
    KC_TRY(kc_tmp_alloc(stats, 8 * 4, s));
    KC_HIP(hipMemsetAsync(stats.p, 0, 8 * 4, s));
    const float *pr = nullptr;
    float promote = 3.0e38f;
    if (policy == KC_SCHED_LEARNED) {
        if (!g->mlp_loaded) return kc_fail(KC_ESTATE, "learned schedule requested but no MLP weights are loaded");
        KC_TRY(kc_tmp_alloc(pred, (size_t)n * 4, s));
        KC_TRY(kc_predict_work(g, pred.as<float>(), s));
        pr = pred.as<float>();
        const char *pe = getenv("KC_PROMOTE_LOGWORK");
        promote = pe ? (float)atof(pe) : 9.0f;
    }
    hipLaunchKernelGGL(k_bin, dim3(grid_for(n)), dim3(T), 0, s, (const uint64_t *)g->optr, n, k, d_lds_max, pr,
                       promote, keys.as<uint64_t>(), flag.as<uint32_t>(), stats.as<uint32_t>(),
                       stats.as<uint32_t>() + 4);
    KC_HIP(hipGetLastError());
    KC_TRY(kc_scan_excl_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), n, nullptr, s));
    uint32_t h_stats[8];
    KC_HIP(hipMemcpyAsync(h_stats, stats.p, sizeof(h_stats), hipMemcpyDeviceToHost, s));
    KC_HIP(hipStreamSynchronize(s));
    const uint32_t total = h_stats[0] + h_stats[1] + h_stats[2];
    for (int t = 0; t < 3; ++t) {
        q.count[t] = h_stats[t];
        q.max_d[t] = h_stats[4 + t];
    }
    q.offset[0] = 0;
    q.offset[1] = q.count[0];
    q.offset[2] = q.count[0] + q.count[1];
    q.offset[3] = total;
    if (total == 0) return KC_OK;
    KC_TRY(kc_tmp_alloc(keys2, (size_t)total * 8, s));
    KC_TRY(kc_tmp_alloc(tmp, (size_t)total * 8, s));
    hipLaunchKernelGGL(k_compact_keys, dim3(grid_for(n)), dim3(T), 0, s, (const uint64_t *)keys.as<uint64_t>(),
                       (const uint32_t *)flag.as<uint32_t>(), (const uint32_t *)pos.as<uint32_t>(), n,
                       keys2.as<uint64_t>());
    KC_HIP(hipGetLastError());
    KC_TRY(kc_radix_sort_u64(keys2.as<uint64_t>(), tmp.as<uint64_t>(), total, 32, 64, s));
    KC_TRY(kc_tmp_alloc(q.buf, (size_t)total * 4, s));
    hipLaunchKernelGGL(k_queue_from_keys, dim3(grid_for(total)), dim3(T), 0, s,
                       (const uint64_t *)keys2.as<uint64_t>(), total, q.buf.as<uint32_t>());
    KC_HIP(hipGetLastError());
    return KC_OK;
}
