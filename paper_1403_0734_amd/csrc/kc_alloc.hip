// Caching device allocator for the library's buffers.
//
// The stream-ordered pool allocator costs hundreds of microseconds to
// milliseconds per call on large buffers while the device may sit idle; the
// counting path allocates and frees the same sizes on every call, so freed
// blocks are kept and handed out again:
//   * a block freed on stream s may still be read by work queued on s, so it is
//     reusable at once only by later work on the same stream (stream order);
//   * after a host synchronisation of s (kc_sync) all of s's freed blocks are
//     idle and reusable on any stream of the device.
// Sizes are rounded up to a bucket (powers of two up to 1 MiB, eighths of a
// power of two beyond) and a block is reused for its exact bucket only.  When
// the cached bytes of a device exceed a quarter of its memory, or an allocation
// fails, the device is synchronised and every cached block is released.
#include <map>
#include <mutex>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "kc_internal.h"

namespace {

struct Block {
    size_t bytes;
    int device;
};

std::mutex g_mu;
std::unordered_map<void *, Block> g_live;                                       // every block handed out or cached
std::map<std::tuple<int, hipStream_t, size_t>, std::vector<void *>> g_pending;  // freed on a stream
std::map<std::pair<int, size_t>, std::vector<void *>> g_idle;                   // reusable on any stream
size_t g_cached[64] = {0};
size_t g_limit[64] = {0};

size_t bucket(size_t b) {
    if (b <= 256) return 256;
    if (b <= ((size_t)1 << 20)) {
        size_t p = 512;
        while (p < b) p <<= 1;
        return p;
    }
    const int lg = 63 - __builtin_clzll((unsigned long long)b);
    const size_t g = (size_t)1 << (lg - 3);
    return (b + g - 1) & ~(g - 1);
}

bool pop(std::vector<void *> &v, void **p) {
    if (v.empty()) return false;
    *p = v.back();
    v.pop_back();
    return true;
}

// Release every cached block of a device (caller holds g_mu).
void release_device(int dev) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    for (auto it = g_pending.begin(); it != g_pending.end();) {
        if (std::get<0>(it->first) == dev) {
            for (void *p : it->second) {
                (void)hipFree(p);
                g_live.erase(p);
            }
            it = g_pending.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = g_idle.begin(); it != g_idle.end();) {
        if (it->first.first == dev) {
            for (void *p : it->second) {
                (void)hipFree(p);
                g_live.erase(p);
            }
            it = g_idle.erase(it);
        } else {
            ++it;
        }
    }
    g_cached[dev] = 0;
    (void)hipSetDevice(cur);
}

}  // namespace

kc_status kc_cache_alloc(void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    int dev = 0;
    KC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return kc_fail(KC_EDEVICE, "device ordinal %d out of range", dev);
    const size_t sz = bucket(bytes ? bytes : 1);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto pi = g_pending.find(std::make_tuple(dev, s, sz));
        if (pi != g_pending.end() && pop(pi->second, p)) {
            g_cached[dev] -= sz;
            return KC_OK;
        }
        auto ii = g_idle.find(std::make_pair(dev, sz));
        if (ii != g_idle.end() && pop(ii->second, p)) {
            g_cached[dev] -= sz;
            return KC_OK;
        }
    }
    hipError_t e = hipMalloc(p, sz);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(g_mu);
        release_device(dev);
        e = hipMalloc(p, sz);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        return kc_hip_fail(e, "hipMalloc", __FILE__, __LINE__);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_live[*p] = Block{sz, dev};
    return KC_OK;
}

void kc_cache_free(void *p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;  // not ours
    const Block b = it->second;
    g_pending[std::make_tuple(b.device, s, b.bytes)].push_back(p);
    g_cached[b.device] += b.bytes;
    if (!g_limit[b.device]) {
        size_t fr = 0, tot = 0;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(b.device);
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = (size_t)16 << 30;
        (void)hipSetDevice(cur);
        g_limit[b.device] = tot / 4;
    }
    if (g_cached[b.device] > g_limit[b.device]) release_device(b.device);
}

kc_status kc_sync(hipStream_t s) {
    KC_HIP(hipStreamSynchronize(s));
    int dev = 0;
    KC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_pending.begin(); it != g_pending.end();) {
        // a stream belongs to one device; the null stream is the current device's
        if (std::get<1>(it->first) == s && (s != nullptr || std::get<0>(it->first) == dev)) {
            auto &dst = g_idle[std::make_pair(std::get<0>(it->first), std::get<2>(it->first))];
            dst.insert(dst.end(), it->second.begin(), it->second.end());
            it = g_pending.erase(it);
        } else {
            ++it;
        }
    }
    return KC_OK;
}
