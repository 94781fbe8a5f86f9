// Ingest (simple graph + degrees) and the degree-ordered orientation.
//
// Ingest (Section 2: the input is an edge set whose endpoints carry degrees):
//   every input edge (u, v), u != v, becomes the undirected key (min, max); a
//   radix sort and a neighbour-difference flag leave each edge once; d(x) counts
//   the edges at x.  The symmetric CSR of the simple graph is built from the
//   unique edges only when it is asked for (kc_get_csr): the count never reads it.
// Orientation (Section 2 total order; Algorithm 1 round 1):
//   nodes are sorted by (d(u), u) and relabelled by position (rank); every edge
//   becomes the rank pair (lower rank, higher rank), i.e. it leaves its endpoint
//   that is smaller in the paper's order; a second radix sort of those pairs is
//   the oriented CSR, out-lists ascending in rank, i.e. in the paper's order.
#include "kc_internal.h"

namespace {

constexpr int T = 256;

inline unsigned grid_for(size_t n, int per = T) { return (unsigned)((n + per - 1) / per); }

// undirected key (min << B) | max of an input edge; self-loops and bad ids map to the sentinel
__global__ void k_make_keys(const uint32_t *src, const uint32_t *dst, size_t m_in, uint32_t n, int B,
                            uint64_t sentinel, uint64_t *keys, uint32_t *err) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m_in) return;
    const uint32_t u = src[i], v = dst[i];
    uint64_t k = sentinel;
    if (u >= n || v >= n) {
        atomicOr(err, 1u);
    } else if (u != v) {
        const uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
        k = ((uint64_t)lo << B) | hi;
    }
    keys[i] = k;
}

// Degrees without global atomics.  d(x) = (edges whose smaller end is x) + (edges
// whose larger end is x).  The first term is a run length of the unique edges,
// which are sorted by their smaller end: a binary search per node.  For the
// second, a copy of the edges is ordered by the top bits of the larger end
// (radix passes from bit RB up), so the edges whose larger end falls in one range
// of 2^RB nodes are contiguous; one block counts each range in LDS.
constexpr int DEG_RANGE_BITS_MAX = 15;  // at most 2^15 LDS counters (128 KB) per block

__device__ __forceinline__ size_t lower_bound_key(const uint64_t *keys, size_t m, uint64_t v, uint64_t mask, int sh) {
    size_t lo = 0, len = m;
    while (len > 0) {
        const size_t half = len >> 1;
        if (((keys[lo + half] & mask) >> sh) < v) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// deg[x] = number of edges with smaller end x: the run of keys from x's first to
// x+1's first.  One search per node: the start of x's run is the lane below's end
// (lane 0 searches it too).
__global__ void k_deg_low_end(const uint64_t *ukeys, size_t m, int B, uint32_t n, uint32_t *deg) {
    const size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63u;
    const size_t b = x < n ? lower_bound_key(ukeys, m, (uint64_t)x + 1, ~0ull, B) : 0;
    const unsigned long long below = __shfl_up((unsigned long long)b, 1, 64);
    size_t a = (size_t)below;
    if (lane == 0 && x < n) a = lower_bound_key(ukeys, m, (uint64_t)x, ~0ull, B);
    if (x < n) deg[x] = (uint32_t)(b - a);
}

// deg[x] += number of edges with larger end x, for the range of block blockIdx.x.
// One block per range (2^RB nodes, as few as 256 blocks): 1024 threads, so that
// enough loads are in flight on each compute unit.
constexpr unsigned DEG_HIGH_THREADS = 1024;
__global__ void __launch_bounds__(DEG_HIGH_THREADS) k_deg_high_end(const uint64_t *bykeys, size_t m, uint64_t mask, int RB,
                                                      uint32_t n, uint32_t *deg) {
    extern __shared__ uint32_t cnt[];
    const uint32_t range = 1u << RB;
    const uint64_t r = blockIdx.x;
    for (uint32_t t = threadIdx.x; t < range; t += blockDim.x) cnt[t] = 0;
    const size_t a = lower_bound_key(bykeys, m, r, mask, RB);
    const size_t b = lower_bound_key(bykeys, m, r + 1, mask, RB);
    __syncthreads();
    for (size_t e = a + threadIdx.x; e < b; e += blockDim.x)
        atomicAdd(&cnt[(uint32_t)(bykeys[e] & mask) & (range - 1)], 1u);
    __syncthreads();
    const uint64_t base = r << RB;
    for (uint32_t t = threadIdx.x; t < range; t += blockDim.x)
        if (base + t < n) deg[base + t] += cnt[t];
}

// both directions of every unique edge, for the symmetric CSR
__global__ void k_sym_keys(const uint64_t *ukeys, size_t m, int B, uint64_t mask, uint64_t *keys) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint64_t k = ukeys[e];
    keys[2 * e] = k;
    keys[2 * e + 1] = ((k & mask) << B) | (k >> B);
}

// flag[i] = 1 for the first copy of each key that is not the sentinel
__global__ void k_unique_flags(const uint64_t *keys, size_t N, uint64_t sentinel, uint32_t *flag) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint64_t k = keys[i];
    flag[i] = (k != sentinel && (i == 0 || keys[i - 1] != k)) ? 1u : 0u;
}

__global__ void k_compact_u64(const uint64_t *in, const uint32_t *flag, const uint32_t *pos, size_t N,
                              uint64_t *out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (flag[i]) out[pos[i]] = in[i];
}

// Row pointers of a CSR given its keys sorted by row (row = key >> B):
// rowptr[r] = first position whose row is >= r (a binary search per row, so
// that runs of empty rows cost nothing extra), rowptr[n] = M.
__global__ void k_rowptr(const uint64_t *keys, size_t M, int B, uint32_t n, uint64_t *rowptr) {
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    const uint64_t key = (uint64_t)r << B;
    size_t lo = 0, len = M;
    while (len > 0) {
        const size_t half = len >> 1;
        if (keys[lo + half] < key) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    rowptr[r] = lo;
}

__global__ void k_fill_u64(uint64_t *p, size_t n, uint64_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_low_bits(const uint64_t *keys, size_t M, uint64_t mask, uint32_t *out) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < M) out[p] = (uint32_t)(keys[p] & mask);
}

// Row lengths (optional) and their maximum (optional): grid-stride, one atomic per block.
__global__ void k_row_lengths(const uint64_t *rowptr, uint32_t n, uint32_t *len, uint32_t *maxlen) {
    __shared__ uint32_t s_max[T / 64];
    uint32_t mx = 0;
    for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (size_t)gridDim.x * blockDim.x) {
        const uint32_t l = (uint32_t)(rowptr[x + 1] - rowptr[x]);
        if (len) len[x] = l;
        mx = l > mx ? l : mx;
    }
    if (maxlen) {
        mx = kc_wave_max_u32(mx);
        if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < T / 64; ++w) mx = s_max[w] > mx ? s_max[w] : mx;
            atomicMax(maxlen, mx);
        }
    }
}
constexpr unsigned ROWLEN_BLOCKS = 1024;
inline unsigned rowlen_grid(uint32_t n) {
    const unsigned g = grid_for(n);
    return g < ROWLEN_BLOCKS ? (g ? g : 1u) : ROWLEN_BLOCKS;
}

// node key (d(x), x): the paper's order as one integer
__global__ void k_node_keys(const uint32_t *deg, uint32_t n, int B, uint64_t *keys) {
    const size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) keys[x] = ((uint64_t)deg[x] << B) | x;
}

__global__ void k_ranks(const uint64_t *sorted, uint32_t n, uint64_t mask, uint32_t *rank2id, uint32_t *id2rank) {
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t id = (uint32_t)(sorted[r] & mask);
    rank2id[r] = id;
    id2rank[id] = (uint32_t)r;
}

// the edge from its endpoint of lower rank (smaller (d, id)) to the other, in rank space
__global__ void k_orient_pairs(const uint64_t *ukeys, size_t m, int B, uint64_t mask, const uint32_t *id2rank,
                               uint64_t *okeys) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint64_t k = ukeys[e];
    const uint32_t ru = id2rank[k >> B], rv = id2rank[k & mask];
    okeys[e] = ru < rv ? (((uint64_t)ru << B) | rv) : (((uint64_t)rv << B) | ru);
}

kc_status degrees(const uint64_t *ukeys, size_t M, int B, uint64_t mask, uint32_t n, uint32_t *deg,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_deg_low_end, dim3(grid_for(n)), dim3(T), 0, s, ukeys, M, B, n, deg);
    KC_HIP(hipGetLastError());
    // p radix passes over the larger end's bits [RB, B), RB = B - 8p, until a range
    // of 2^RB nodes fits the LDS counters
    int p = 0;
    while (B - 8 * p > DEG_RANGE_BITS_MAX) ++p;
    if (p == 0 && B > 8 && M > 65536) p = 1;  // many edges: spread them over 256 ranges
    const int RB = B - 8 * p > 0 ? B - 8 * p : 0;
    const uint64_t *by = ukeys;
    kc_tmp copy, tmp;
    if (RB < B && p == 1) {
        // one pass reads ukeys and writes tmp only: no copy needed
        KC_TRY(kc_tmp_alloc(tmp, M * 8, s));
        uint64_t *sorted = nullptr;
        KC_TRY(kc_radix_sort_u64(const_cast<uint64_t *>(ukeys), tmp.as<uint64_t>(), M, RB, B, s, &sorted));
        by = sorted;
    } else if (RB < B) {
        KC_TRY(kc_tmp_alloc(copy, M * 8, s));
        KC_TRY(kc_tmp_alloc(tmp, M * 8, s));
        KC_HIP(hipMemcpyAsync(copy.p, ukeys, M * 8, hipMemcpyDeviceToDevice, s));
        KC_TRY(kc_radix_sort_u64(copy.as<uint64_t>(), tmp.as<uint64_t>(), M, RB, B, s));
        by = copy.as<uint64_t>();
    }
    const uint64_t ranges = (((uint64_t)n - 1) >> RB) + 1;
    const size_t lds = (size_t)4 << RB;
    (void)hipFuncSetAttribute((const void *)&k_deg_high_end, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_deg_high_end, dim3((unsigned)ranges), dim3(DEG_HIGH_THREADS), lds, s, by, M, mask, RB, n,
                       deg);
    KC_HIP(hipGetLastError());
    return KC_OK;
}

kc_status rows_from_sorted(const uint64_t *keys, size_t M, int B, uint32_t n, uint64_t *rowptr, hipStream_t s) {
    if (M == 0) {
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_for((size_t)n + 1)), dim3(T), 0, s, rowptr, (size_t)n + 1, 0ull);
    } else {
        hipLaunchKernelGGL(k_rowptr, dim3(grid_for((size_t)n + 1)), dim3(T), 0, s, keys, M, B, n, rowptr);
    }
    KC_HIP(hipGetLastError());
    return KC_OK;
}

}  // namespace

kc_status kc_canonicalise(kc_graph *g, const uint32_t *d_src, const uint32_t *d_dst) {
    hipStream_t s = g->stream;
    const uint32_t n = g->n;
    const int B = g->idbits;
    const size_t N = (size_t)g->m_in;
    const uint64_t mask = (B >= 64) ? ~0ull : ((1ull << B) - 1ull);
    const uint64_t sentinel = (2 * B >= 64) ? ~0ull : ((1ull << (2 * B)) - 1ull);

    KC_TRY(kc_dev_alloc((void **)&g->deg, (size_t)n * sizeof(uint32_t), s));
    KC_HIP(hipMemsetAsync(g->deg, 0, (size_t)n * sizeof(uint32_t), s));
    kc_tmp keys, tmp, flag, pos, err, total;
    KC_TRY(kc_tmp_alloc(err, sizeof(uint32_t) * 2, s));
    KC_TRY(kc_tmp_alloc(total, sizeof(uint32_t) * 2, s));
    KC_HIP(hipMemsetAsync(err.p, 0, sizeof(uint32_t) * 2, s));
    uint32_t M = 0;
    if (N > 0) {
        KC_TRY(kc_tmp_alloc(keys, N * sizeof(uint64_t), s));
        KC_TRY(kc_tmp_alloc(tmp, N * sizeof(uint64_t), s));
        hipLaunchKernelGGL(k_make_keys, dim3(grid_for(N)), dim3(T), 0, s, d_src, d_dst, N, n, B, sentinel,
                           keys.as<uint64_t>(), err.as<uint32_t>());
        KC_HIP(hipGetLastError());
        uint64_t *sk = nullptr;  // the sorted keys (either buffer)
        KC_TRY(kc_radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), N, 0, 2 * B, s, &sk));
        KC_TRY(kc_tmp_alloc(flag, N * sizeof(uint32_t), s));
        KC_TRY(kc_tmp_alloc(pos, N * sizeof(uint32_t), s));
        hipLaunchKernelGGL(k_unique_flags, dim3(grid_for(N)), dim3(T), 0, s, (const uint64_t *)sk, N, sentinel,
                           flag.as<uint32_t>());
        KC_HIP(hipGetLastError());
        KC_TRY(kc_scan_excl_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), N, total.as<uint32_t>(), s));
        uint32_t *h = (uint32_t *)kc_pinned_scratch();
        KC_HIP(hipMemcpyAsync(h, err.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        KC_HIP(hipMemcpyAsync(h + 1, total.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        KC_TRY(kc_sync(s));
        if (h[0]) return kc_fail(KC_EINVAL, "an edge endpoint is >= n (%u)", n);
        M = h[1];
        // the unique edges stay on the handle: orientation and the symmetric CSR read them
        KC_TRY(kc_dev_alloc((void **)&g->ukeys, (size_t)(M ? M : 1) * sizeof(uint64_t), s));
        hipLaunchKernelGGL(k_compact_u64, dim3(grid_for(N)), dim3(T), 0, s, (const uint64_t *)sk,
                           flag.as<uint32_t>(), pos.as<uint32_t>(), N, g->ukeys);
        KC_HIP(hipGetLastError());
        if (M) KC_TRY(degrees(g->ukeys, M, B, mask, n, g->deg, s));
    }
    g->m = M;
    return KC_OK;  // the caller synchronises
}

// The symmetric CSR (rowptr, col) of the simple graph, built on first request.
kc_status kc_build_csr(kc_graph *g) {
    if (g->rowptr) return KC_OK;
    hipStream_t s = g->stream;
    const uint32_t n = g->n;
    const int B = g->idbits;
    const uint64_t mask = (B >= 64) ? ~0ull : ((1ull << B) - 1ull);
    const size_t M2 = 2 * (size_t)g->m;
    KC_TRY(kc_dev_alloc((void **)&g->rowptr, ((size_t)n + 1) * sizeof(uint64_t), s));
    KC_TRY(kc_dev_alloc((void **)&g->col, (size_t)(M2 ? M2 : 1) * sizeof(uint32_t), s));
    kc_tmp keys, tmp;
    if (M2) {
        KC_TRY(kc_tmp_alloc(keys, M2 * sizeof(uint64_t), s));
        KC_TRY(kc_tmp_alloc(tmp, M2 * sizeof(uint64_t), s));
        hipLaunchKernelGGL(k_sym_keys, dim3(grid_for(g->m)), dim3(T), 0, s, (const uint64_t *)g->ukeys, (size_t)g->m,
                           B, mask, keys.as<uint64_t>());
        KC_HIP(hipGetLastError());
        KC_TRY(kc_radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), M2, 0, 2 * B, s));
        hipLaunchKernelGGL(k_low_bits, dim3(grid_for(M2)), dim3(T), 0, s, (const uint64_t *)keys.as<uint64_t>(), M2,
                           mask, g->col);
        KC_HIP(hipGetLastError());
    }
    KC_TRY(rows_from_sorted(keys.as<uint64_t>(), M2, B, n, g->rowptr, s));
    KC_TRY(kc_sync(s));
    return KC_OK;
}

kc_status kc_orient_impl(kc_graph *g) {
    hipStream_t s = g->stream;
    const uint32_t n = g->n;
    const int B = g->idbits;
    const uint64_t mask = (B >= 64) ? ~0ull : ((1ull << B) - 1ull);

    KC_TRY(kc_dev_alloc((void **)&g->optr, ((size_t)n + 1) * sizeof(uint64_t), s));
    KC_TRY(kc_dev_alloc((void **)&g->ocol, (size_t)(g->m ? g->m : 1) * sizeof(uint32_t), s));
    KC_TRY(kc_dev_alloc((void **)&g->rank2id, (size_t)n * sizeof(uint32_t), s));
    KC_TRY(kc_dev_alloc((void **)&g->id2rank, (size_t)n * sizeof(uint32_t), s));

    // 1. ranks: stable sort of (d(x) << B | x) on the degree bits (ids already ascending)
    kc_tmp nk, nk_tmp;
    KC_TRY(kc_tmp_alloc(nk, (size_t)n * sizeof(uint64_t), s));
    KC_TRY(kc_tmp_alloc(nk_tmp, (size_t)n * sizeof(uint64_t), s));
    hipLaunchKernelGGL(k_node_keys, dim3(grid_for(n)), dim3(T), 0, s, (const uint32_t *)g->deg, n, B,
                       nk.as<uint64_t>());
    KC_HIP(hipGetLastError());
    KC_TRY(kc_radix_sort_u64(nk.as<uint64_t>(), nk_tmp.as<uint64_t>(), n, B, 2 * B, s));
    hipLaunchKernelGGL(k_ranks, dim3(grid_for(n)), dim3(T), 0, s, (const uint64_t *)nk.as<uint64_t>(), n, mask,
                       g->rank2id, g->id2rank);
    KC_HIP(hipGetLastError());

    // 2. every edge once, from its lower-ranked endpoint, in rank space
    kc_tmp okeys, otmp, maxd;
    KC_TRY(kc_tmp_alloc(maxd, sizeof(uint32_t), s));
    KC_HIP(hipMemsetAsync(maxd.p, 0, sizeof(uint32_t), s));
    const size_t m = g->m;
    uint64_t *sorted = nullptr;
    if (m > 0) {
        KC_TRY(kc_tmp_alloc(okeys, m * sizeof(uint64_t), s));
        KC_TRY(kc_tmp_alloc(otmp, m * sizeof(uint64_t), s));
        hipLaunchKernelGGL(k_orient_pairs, dim3(grid_for(m)), dim3(T), 0, s, (const uint64_t *)g->ukeys, m, B, mask,
                           (const uint32_t *)g->id2rank, okeys.as<uint64_t>());
        KC_HIP(hipGetLastError());
        KC_TRY(kc_radix_sort_u64(okeys.as<uint64_t>(), otmp.as<uint64_t>(), m, 0, 2 * B, s, &sorted));
        hipLaunchKernelGGL(k_low_bits, dim3(grid_for(m)), dim3(T), 0, s, (const uint64_t *)sorted, m, mask, g->ocol);
        KC_HIP(hipGetLastError());
    }
    KC_TRY(rows_from_sorted(sorted, m, B, n, g->optr, s));
    hipLaunchKernelGGL(k_row_lengths, dim3(rowlen_grid(n)), dim3(T), 0, s, (const uint64_t *)g->optr, n,
                       (uint32_t *)nullptr, maxd.as<uint32_t>());
    KC_HIP(hipGetLastError());
    uint32_t *h = (uint32_t *)kc_pinned_scratch();
    KC_HIP(hipMemcpyAsync(h, maxd.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    KC_TRY(kc_sync(s));
    g->max_outdeg = h[0];
    g->oriented = 1;
    return KC_OK;
}

