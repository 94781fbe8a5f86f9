// Device-wide primitives: exclusive scan and a stable LSD radix sort of 64-bit
// keys.  Both are HBM-bound passes used by canonicalisation, orientation and
// queue building.
#include "kc_internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Block-wide exclusive scan of one value per thread; returns the block total.
template <typename T>
__device__ T block_excl_scan(T v, T *s_waves, T &total) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    T x = v;
    for (int off = 1; off < 64; off <<= 1) {
        T o = __shfl_up(x, off, 64);
        if (lane >= off) x += o;
    }
    if (lane == 63) s_waves[wave] = x;
    __syncthreads();
    T wbase = 0, tot = 0;
    for (int w = 0; w < SCAN_THREADS / 64; ++w) {
        if (w < wave) wbase += s_waves[w];
        tot += s_waves[w];
    }
    total = tot;
    __syncthreads();
    return wbase + x - v;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const T *in, size_t n, T *partial) {
    __shared__ T s_waves[SCAN_THREADS / 64];
    const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
    T s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j)
        if (base + j < n) s += in[base + j];
    T total;
    (void)block_excl_scan<T>(s, s_waves, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of each tile, offset by the scanned tile partials (may be null).
template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_apply(const T *in, T *out, size_t n, const T *partial_excl,
                                                             T *d_total) {
    __shared__ T s_waves[SCAN_THREADS / 64];
    const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        v[j] = (base + j < n) ? in[base + j] : (T)0;
        s += v[j];
    }
    T total;
    T run = block_excl_scan<T>(s, s_waves, total);
    if (partial_excl) run += partial_excl[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (d_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) *d_total = run;
}

template <typename T>
kc_status scan_excl(const T *in, T *out, size_t n, T *d_total, hipStream_t s) {
    if (n == 0) {
        if (d_total) KC_HIP(hipMemsetAsync(d_total, 0, sizeof(T), s));
        return KC_OK;
    }
    const size_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles == 1) {
        hipLaunchKernelGGL(k_scan_apply<T>, dim3(1), dim3(SCAN_THREADS), 0, s, in, out, n, (const T *)nullptr,
                           d_total);
        KC_HIP(hipGetLastError());
        return KC_OK;
    }
    kc_tmp part, part_x;
    KC_TRY(kc_tmp_alloc(part, tiles * sizeof(T), s));
    KC_TRY(kc_tmp_alloc(part_x, tiles * sizeof(T), s));
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, s, in, n, part.as<T>());
    KC_HIP(hipGetLastError());
    KC_TRY(scan_excl<T>(part.as<T>(), part_x.as<T>(), tiles, (T *)nullptr, s));
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, s, in, out, n,
                       (const T *)part_x.as<T>(), d_total);
    KC_HIP(hipGetLastError());
    return KC_OK;
}

// ----------------------------------------------------------------------------
// Radix sort: 8-bit digits, 256 threads x 16 keys per tile.  Per pass, three
// launches: tile histograms (digit-major), an exclusive scan of each digit's
// row of tile counts (one block per digit, which also writes the digit's
// total), and a stable scatter that scans the 256 digit totals itself.
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

// Lanes whose 8-bit digit equals this lane's (among valid lanes).
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return valid ? peers : 0ull;
}

__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint64_t *keys, size_t n, int shift, uint32_t *hist,
                                                        uint32_t nblocks) {
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        const size_t i = base + (size_t)r * RS_THREADS + threadIdx.x;
        const bool valid = i < n;
        const uint32_t d = valid ? (uint32_t)(keys[i] >> shift) & 255u : 0u;
        const uint64_t peers = match_digit8(d, valid);
        if (valid && (peers & kc_lanemask_lt()) == 0) atomicAdd(&s_h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = s_h[threadIdx.x];
}

// offs[d * nblocks + b] = exclusive scan of hist[d * nblocks + 0 .. nblocks), for the
// digit d of this block; total[d] = the digit's count.
__global__ void __launch_bounds__(RS_THREADS) k_rs_rowscan(const uint32_t *hist, uint32_t *offs, uint32_t nblocks,
                                                           uint32_t *total) {
    __shared__ uint32_t s_wt[RS_THREADS / 64];
    const uint32_t *row = hist + (size_t)blockIdx.x * nblocks;
    uint32_t *orow = offs + (size_t)blockIdx.x * nblocks;
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    const uint32_t per = (nblocks + RS_THREADS - 1) / RS_THREADS;
    const uint32_t b0 = tid * per, b1 = b0 + per < nblocks ? b0 + per : nblocks;
    uint32_t sum = 0;
    for (uint32_t b = b0; b < b1; ++b) sum += row[b];
    const uint32_t inc = kc_wave_incl_u32(sum);
    if ((tid & 63) == 63) s_wt[wave] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (uint32_t w = 0; w < wave; ++w) run += s_wt[w];
    for (uint32_t b = b0; b < b1; ++b) {
        orow[b] = run;
        run += row[b];
    }
    if (tid == RS_THREADS - 1) total[blockIdx.x] = run;
}

// Stable scatter of one tile: keys are first ranked and placed in LDS in digit
// order (tile-local start of each digit from this tile's histogram), then
// written out in that order, so that each digit's keys of the tile leave as
// one contiguous run.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint64_t *in, uint64_t *out, size_t n, int shift,
                                                           const uint32_t *hist, const uint32_t *offs,
                                                           const uint32_t *dtotal, uint32_t nblocks) {
    __shared__ uint64_t s_keys[RS_TILE];
    __shared__ uint32_t s_start[256];  // tile-local first position of each digit
    __shared__ uint32_t s_run[256];    // keys of each digit placed so far
    __shared__ uint32_t s_gbase[256];  // global first position of each digit's run
    __shared__ uint32_t s_w[RS_THREADS / 64][256];
    __shared__ uint32_t s_wt[RS_THREADS / 64];
    __shared__ uint32_t s_dt[RS_THREADS / 64];
    const int tid = threadIdx.x, wave = tid >> 6;
    // tile-local digit starts from this tile's counts; global digit starts from the totals
    const uint32_t c = hist[(size_t)tid * nblocks + blockIdx.x];
    const uint32_t inc = kc_wave_incl_u32(c);
    const uint32_t dt = dtotal[tid];
    const uint32_t dinc = kc_wave_incl_u32(dt);
    if ((tid & 63) == 63) {
        s_wt[wave] = inc;
        s_dt[wave] = dinc;
    }
    s_run[tid] = 0;
    __syncthreads();
    uint32_t before = 0, dbefore = 0;
    for (int w = 0; w < wave; ++w) {
        before += s_wt[w];
        dbefore += s_dt[w];
    }
    s_start[tid] = before + inc - c;
    s_gbase[tid] = dbefore + dinc - dt + offs[(size_t)tid * nblocks + blockIdx.x];
    const size_t base = (size_t)blockIdx.x * RS_TILE;
    uint64_t kk[RS_ITEMS];  // the tile's keys, all loads issued before the ranking
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const size_t i = base + (size_t)r * RS_THREADS + tid;
        kk[r] = i < n ? in[i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const size_t i = base + (size_t)r * RS_THREADS + tid;
        const bool valid = i < n;
        const uint64_t key = kk[r];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
#pragma unroll
        for (int w = 0; w < RS_THREADS / 64; ++w) s_w[w][tid] = 0;
        __syncthreads();
        const uint64_t peers = match_digit8(d, valid);
        const uint64_t lower = peers & kc_lanemask_lt();
        if (valid && lower == 0) s_w[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = s_start[d] + s_run[d] + (uint32_t)__popcll(lower);
            for (int w = 0; w < wave; ++w) off += s_w[w][d];
            s_keys[off] = key;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < RS_THREADS / 64; ++w) add += s_w[w][tid];
        s_run[tid] += add;
    }
    __syncthreads();
    const size_t left = n - base;
    const uint32_t tile_n = left < (size_t)RS_TILE ? (uint32_t)left : (uint32_t)RS_TILE;
    for (uint32_t q = tid; q < tile_n; q += RS_THREADS) {
        const uint64_t key = s_keys[q];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        out[(size_t)s_gbase[d] + (q - s_start[d])] = key;
    }
}

}  // namespace

kc_status kc_scan_excl_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *d_total, hipStream_t s) {
    return scan_excl<uint32_t>(in, out, n, d_total, s);
}
kc_status kc_scan_excl_u64(const uint64_t *in, uint64_t *out, size_t n, uint64_t *d_total, hipStream_t s) {
    return scan_excl<uint64_t>(in, out, n, d_total, s);
}

kc_status kc_radix_sort_u64(uint64_t *keys, uint64_t *tmp, size_t n, int bit_lo, int bit_hi, hipStream_t s,
                            uint64_t **sorted) {
    if (sorted) *sorted = keys;
    if (n <= 1 || bit_hi <= bit_lo) return KC_OK;
    if (n >= (1ull << 32)) return kc_fail(KC_EINVAL, "radix sort of %zu keys exceeds 2^32", n);
    const uint32_t nblocks = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
    kc_tmp hist, offs, dtot;
    KC_TRY(kc_tmp_alloc(hist, (size_t)256 * nblocks * sizeof(uint32_t), s));
    KC_TRY(kc_tmp_alloc(offs, (size_t)256 * nblocks * sizeof(uint32_t), s));
    KC_TRY(kc_tmp_alloc(dtot, 256 * sizeof(uint32_t), s));
    uint64_t *src = keys, *dst = tmp;
    int passes = 0;
    for (int shift = bit_lo; shift < bit_hi; shift += 8, ++passes) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(RS_THREADS), 0, s, (const uint64_t *)src, n, shift,
                           hist.as<uint32_t>(), nblocks);
        KC_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(RS_THREADS), 0, s, (const uint32_t *)hist.as<uint32_t>(),
                           offs.as<uint32_t>(), nblocks, dtot.as<uint32_t>());
        KC_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(RS_THREADS), 0, s, (const uint64_t *)src, dst, n,
                           shift, (const uint32_t *)hist.as<uint32_t>(), (const uint32_t *)offs.as<uint32_t>(),
                           (const uint32_t *)dtot.as<uint32_t>(), nblocks);
        KC_HIP(hipGetLastError());
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    if (sorted) *sorted = src;
    else if (passes & 1) KC_HIP(hipMemcpyAsync(keys, tmp, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    return KC_OK;
}
