// Peak microbenchmarks (include/kc_peaks.h): HBM copy, LDS 128-bit reads, int32
// VALU and 64-bit AND + popcount loops, each timed with HIP events.
#include <hip/hip_runtime.h>

#include "kc_peaks.h"

namespace {

constexpr int T = 256;

// Four 16-byte words per thread per round (four loads in flight), non-temporal.
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(T) k_copy(const v4u *__restrict__ src, v4u *__restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v4u a = __builtin_nontemporal_load(src + i), b = __builtin_nontemporal_load(src + i + stride),
                  c = __builtin_nontemporal_load(src + i + 2 * stride),
                  d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// Each thread reads four 128-bit words of a 16 KB LDS array per round, at
// addresses that move with the round (so the reads stay in the loop) and cover
// all banks; the XOR of everything read is written only when it equals a value
// the host never passes, so the reads cannot be removed.
__global__ void __launch_bounds__(T) k_lds(int reps, uint32_t never, uint32_t *sink) {
    __shared__ uint4 buf[1024];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < 1024; i += T) buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
    __syncthreads();
    uint4 a = make_uint4(0, 0, 0, 0), b = a;
    uint32_t o = 0;
    for (int r = 0; r < reps; r += 4) {
        const uint32_t base = t ^ o;  // < 256
        const uint4 x0 = buf[base], x1 = buf[base + 256], x2 = buf[base + 512], x3 = buf[base + 768];
        a.x ^= x0.x ^ x1.x; a.y ^= x0.y ^ x1.y; a.z ^= x0.z ^ x1.z; a.w ^= x0.w ^ x1.w;
        b.x ^= x2.x ^ x3.x; b.y ^= x2.y ^ x3.y; b.z ^= x2.z ^ x3.z; b.w ^= x2.w ^ x3.w;
        o = (o + 37u) & 255u;
    }
    const uint32_t v = a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w;
    if (v == never) sink[0] = v;
}

// 8 chains of (add, xor): 16 int32 VALU operations per round, independent chains.
__global__ void __launch_bounds__(T) k_valu(int reps, uint32_t seed, uint32_t never, uint32_t *sink) {
    uint32_t x[8], y[8];
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        x[c] = t * (2u * c + 1u) + seed;
        y[c] = seed ^ (c * 0x9E3779B9u);
    }
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            x[c] = x[c] + y[c];
            y[c] = y[c] ^ x[c];
        }
    }
    uint32_t v = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) v ^= x[c] ^ y[c];
    if (v == never) sink[0] = v;
}

// 8 independent accumulations of popcount(a & b) over 64-bit words (the counting
// kernels' intersection step); the words change each round so nothing is hoisted.
__global__ void __launch_bounds__(T) k_andpop(int reps, uint64_t seed, uint32_t never, uint32_t *sink) {
    uint64_t a[8];
    uint32_t acc[8];
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        a[c] = (t + 1) * (0x9E3779B97F4A7C15ull + (uint64_t)c) ^ seed;
        acc[c] = 0;
    }
    uint64_t b = seed | 1ull;
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] += (uint32_t)__popcll(a[c] & b);
        b = (b << 1) | (b >> 63);
    }
    uint32_t v = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) v += acc[c];
    if (v == never) sink[0] = v;
}

template <class F>
int timed(int32_t iters, hipStream_t s, float *ms, F launch) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        launch();  // warm-up
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int i = 0; e == hipSuccess && i < iters; ++i) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return (int)e;
    *ms = t / (float)iters;
    return 0;
}

struct Sink {
    uint32_t *p = nullptr;
    ~Sink() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" int kcp_hbm_copy(const void *src, void *dst, size_t bytes, int32_t iters, void *hip_stream, float *ms,
                            double *work) {
    if (!src || !dst || !ms || !work || iters < 1 || bytes == 0 || bytes % 16 ||
        ((uintptr_t)src | (uintptr_t)dst) % 16)
        return -1;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t n = bytes / 16;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const unsigned blocks = (unsigned)cus * 16u;
    *work = 2.0 * (double)bytes;
    return timed(iters, s, ms, [&]() {
        hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(T), 0, s, (const v4u *)src, (v4u *)dst, n);
    });
}

extern "C" int kcp_lds_read(int32_t blocks, int32_t reps, int32_t iters, void *hip_stream, float *ms, double *work) {
    if (blocks < 1 || reps < 4 || iters < 1 || !ms || !work) return -1;
    hipStream_t s = (hipStream_t)hip_stream;
    Sink sink;
    hipError_t e = hipMalloc((void **)&sink.p, 4);
    if (e != hipSuccess) return (int)e;
    const int r = reps & ~3;
    *work = (double)blocks * T * r * 16.0;
    return timed(iters, s, ms, [&]() { hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(T), 0, s, r, 0xDEADBEEFu, sink.p); });
}

extern "C" int kcp_valu_int32(int32_t blocks, int32_t reps, int32_t iters, void *hip_stream, float *ms, double *work) {
    if (blocks < 1 || reps < 1 || iters < 1 || !ms || !work) return -1;
    hipStream_t s = (hipStream_t)hip_stream;
    Sink sink;
    hipError_t e = hipMalloc((void **)&sink.p, 4);
    if (e != hipSuccess) return (int)e;
    *work = (double)blocks * T * reps * 16.0;
    return timed(iters, s, ms, [&]() {
        hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(T), 0, s, reps, 12345u, 0xDEADBEEFu, sink.p);
    });
}

extern "C" int kcp_and_popcount(int32_t blocks, int32_t reps, int32_t iters, void *hip_stream, float *ms,
                                double *work) {
    if (blocks < 1 || reps < 1 || iters < 1 || !ms || !work) return -1;
    hipStream_t s = (hipStream_t)hip_stream;
    Sink sink;
    hipError_t e = hipMalloc((void **)&sink.p, 4);
    if (e != hipSuccess) return (int)e;
    *work = (double)blocks * T * reps * 8.0;
    return timed(iters, s, ms, [&]() {
        hipLaunchKernelGGL(k_andpop, dim3(blocks), dim3(T), 0, s, reps, 0x243F6A8885A308D3ull, 0xFFFFFFFFu, sink.p);
    });
}
