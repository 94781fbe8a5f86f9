// Exact counts for callers that cannot allocate device memory.
//
// kc_count_noalloc runs the same counting kernels as kc_count on a handle that an
// earlier kc_count has prepared (degree queue, staged G+(u) cache).  The per-call
// scratch that kc_count takes from the caching allocator (the result block with
// its queue counters and partial totals, and the global-memory slices of the
// scratch tier) comes instead from one file-scope device array per GPU.  The
// call allocates nothing, synchronises nothing and reads nothing back: q_k and
// the overflow flag are written to caller device memory, ordered on the handle's
// stream.
#include <mutex>

#include "kc_internal.h"

namespace {

// 64 MiB per GPU: the result block (rounded up to 256-byte words) and the slices
// of the scratch tier.  One slice holds the packed bitmap of one root, about
// d^2 / 16 bytes, so out-degrees up to about 32000 fit.
constexpr size_t NOALLOC_BYTES = 64ull << 20;
constexpr size_t NOALLOC_WORDS = NOALLOC_BYTES / 8;
constexpr size_t NOALLOC_RES_WORDS = (KC_RES_WORDS + 31) / 32 * 32;

}  // namespace

static __device__ __align__(256) uint64_t scratch[NOALLOC_WORDS];

namespace {

// Device address of `scratch` on each GPU, looked up once per device with that
// device current.  Host code uses only these addresses: the array's name is a
// host-side stand-in.
std::mutex g_mu;
uint64_t *g_addr[64] = {nullptr};

kc_status scratch_address(int device, uint64_t **out) {
    if (device < 0 || device >= 64) return kc_fail(KC_EINVAL, "device %d outside [0, 64)", device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[device]) {
        int cur = -1;
        KC_HIP(hipGetDevice(&cur));
        if (cur != device) KC_HIP(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) KC_HIP(hipSetDevice(cur));
        if (e != hipSuccess) return kc_hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        if (!p) return kc_fail(KC_EDEVICE, "no device address for the scratch array");
        g_addr[device] = static_cast<uint64_t *>(p);
    }
    *out = g_addr[device];
    return KC_OK;
}

// out[0] = the total, out[1] = 1 when a sum overflowed
__global__ void k_result_out(const uint64_t *res, uint64_t *out) {
    if (threadIdx.x == 0) {
        out[0] = res[0];
        out[1] = res[1] != 0 ? 1ull : 0ull;
    }
}

}  // namespace

extern "C" kc_status kc_count_noalloc(const kc_graph *g, int32_t k, uint64_t *dev_out) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (!dev_out) return kc_fail(KC_EINVAL, "dev_out is NULL");
    if (k < 3 || k > KC_KMAX) return kc_fail(KC_EINVAL, "k=%d outside [3, %d]", k, KC_KMAX);
    if (!g->oriented) return kc_fail(KC_ESTATE, "kc_orient has not been called");
    uint64_t *base = nullptr;
    KC_TRY(scratch_address(g->device, &base));
    hipStream_t s = g->stream;
    int wd = kc_tuning_now().wave_dmax;
    wd = wd < 1 ? 1 : (wd > 64 ? 64 : wd);
    // the handle's degree queue and work items as they are (KC_ESTATE if not built)
    kc_queue q;
    KC_TRY(kc_build_queue(g, k, KC_SCHED_DEGREE, kc_lds_dcap(g->device, k), q, /*no_alloc=*/true));
    // scratch-tier slices after the result block, as many as fit (at most one per CU)
    size_t slice_words = 0;
    uint32_t blocks = 0;
    if (q.count[2]) {
        slice_words = kc_scratch_slice_words(q.max_d[2], k);
        const size_t fit = (NOALLOC_WORDS - NOALLOC_RES_WORDS) / slice_words;
        if (fit == 0)
            return kc_fail(KC_EINVAL, "out-degree %u needs a %zu-byte scratch slice; the no-alloc scratch holds %zu",
                           q.max_d[2], slice_words * 8, (size_t)(NOALLOC_WORDS - NOALLOC_RES_WORDS) * 8);
        int cus = 0;
        KC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
        blocks = q.count[2];
        if (cus > 0 && blocks > (uint32_t)cus) blocks = (uint32_t)cus;
        if (blocks > fit) blocks = (uint32_t)fit;
    }
    kc_count_args a;
    a.k = k;
    a.cached = g->staged == 1 && g->stage_wd == wd;
    uint64_t *res = base;
    KC_TRY(kc_count_launch(g, q, a, res, nullptr, 0, nullptr, base + NOALLOC_RES_WORDS, slice_words, blocks, s,
                           nullptr, false));
    hipLaunchKernelGGL(k_result_out, dim3(1), dim3(64), 0, s, (const uint64_t *)res, dev_out);
    KC_HIP(hipGetLastError());
    return KC_OK;
}
