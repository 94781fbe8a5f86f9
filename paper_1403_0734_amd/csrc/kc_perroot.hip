// Per-root counts and per-root work, and the batch entry point.
#include "kc_internal.h"

namespace {
constexpr int T = 256;
inline unsigned grid_for(size_t n) { return (unsigned)((n + T - 1) / T); }

// work[id] = |Gamma+(u)|: the first-level intersections of the count
__global__ void k_outdeg_by_id(const uint64_t *optr, const uint32_t *rank2id, uint32_t n, uint64_t *work) {
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) work[rank2id[r]] = optr[r + 1] - optr[r];
}

__global__ void k_add_checked(uint64_t *acc, const uint64_t *x, uint32_t n, uint32_t *ovf) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t a = acc[i], b = x[i], s = a + b;
    if (s < a) atomicOr(ovf, 1u);
    acc[i] = s;
}
}  // namespace

extern "C" kc_status kc_count_per_root(const kc_graph *g, int32_t k, uint64_t *dev_counts, uint64_t *dev_work) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (!dev_counts) return kc_fail(KC_EINVAL, "dev_counts is NULL");
    if (k < 3 || k > KC_KMAX) return kc_fail(KC_EINVAL, "k=%d outside [3, %d]", k, KC_KMAX);
    if (!g->oriented) return kc_fail(KC_ESTATE, "kc_orient has not been called");
    hipStream_t s = g->stream;
    kc_count_args a;
    a.k = k;
    a.policy = g->policy;
    a.per_root = dev_counts;
    uint64_t total = 0;
    int ovf = 0;
    KC_TRY(kc_count_impl(g, a, &total, &ovf));
    if (ovf) return kc_fail(KC_EOVERFLOW, "q_%d >= 2^64", k);
    if (dev_work) {
        // W(u, k) = sum_{l=1}^{k-2} (l-cliques of G+(u)): l = 1 is |Gamma+(u)|, and the
        // l-cliques of G+(u) are the per-root counts at clique size l + 1.
        hipLaunchKernelGGL(k_outdeg_by_id, dim3(grid_for(g->n)), dim3(T), 0, s, (const uint64_t *)g->optr,
                           (const uint32_t *)g->rank2id, g->n, dev_work);
        KC_HIP(hipGetLastError());
        if (k >= 4) {
            kc_tmp tmp, flag;
            KC_TRY(kc_tmp_alloc(tmp, (size_t)g->n * 8, s));
            KC_TRY(kc_tmp_alloc(flag, 4, s));
            KC_HIP(hipMemsetAsync(flag.p, 0, 4, s));
            for (int l = 2; l <= k - 2; ++l) {
                kc_count_args b = a;
                b.k = l + 1;
                b.per_root = tmp.as<uint64_t>();
                KC_TRY(kc_count_impl(g, b, &total, &ovf));
                if (ovf) return kc_fail(KC_EOVERFLOW, "work label overflows");
                hipLaunchKernelGGL(k_add_checked, dim3(grid_for(g->n)), dim3(T), 0, s, dev_work,
                                   (const uint64_t *)tmp.as<uint64_t>(), g->n, flag.as<uint32_t>());
                KC_HIP(hipGetLastError());
            }
            uint32_t *h = (uint32_t *)kc_pinned_scratch();
            KC_HIP(hipMemcpyAsync(h, flag.p, 4, hipMemcpyDeviceToHost, s));
            KC_TRY(kc_sync(s));
            if (h[0]) return kc_fail(KC_EOVERFLOW, "work label overflows");
        }
    }
    KC_TRY(kc_sync(s));
    return KC_OK;
}
