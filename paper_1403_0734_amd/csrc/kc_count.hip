// Per-root (k-1)-clique counting in G+(u) and the global reduction.
//
// Section 3, Algorithm 1 (rounds 2 and 3) and Theorem 1: every k-clique is
// counted once, by its smallest node u in the (degree, label) order, as a
// (k-1)-clique of the subgraph G+(u) induced by the high-neighbourhood Gamma+(u).
// Instead of emitting 2-paths and shuffling them (the MapReduce rounds), each
// root pulls its sub-problem:
//
//   staging  For Gamma+(u) = (a_0 < ... < a_{d-1}) (rank order = the paper's
//            order), bit j of row i is set iff a_j is in Gamma+(a_i).  Only
//            j > i can be set, so rows are upper-triangular.  Every out-list
//            Gamma+(a_i) is read once and each id is looked up in Gamma+(u)
//            by binary search (this is the wedge work of round 2).
//   count    cnt(P, 1) = |P|, cnt(P, r) = sum_{v in P} cnt(P n row_v, r - 1),
//            with P a bit set; q_{u,k-1} = cnt({0..d-1}, k-1) (round 3).
//   colour   Section 6 (cFFF_k): with per-root colours, bit (i, j) is kept only
//            when a_i and a_j share their colour; with one global colouring,
//            Gamma+(u) is first cut to the nodes that share u's colour.
//
// Tiers (by out-degree d = |Gamma+(u)|):
//   wave       d <= 64: one wave per root, one 64-bit row per node held in LDS;
//              the count runs as a per-lane depth-first state machine over the
//              edges (i, j) of G+(u), refilling lanes from a wave-local queue.
//   workgroup  64 < d <= D_LDS: one workgroup per root, packed upper-triangular
//              bitmap in LDS; waves take first-level nodes, lanes span words.
//   scratch    d > D_LDS: as workgroup, bitmap in a global-memory slice.
// Every count is an exact uint64; sums are carry-checked.
#include "kc_internal.h"

namespace {

constexpr int WG = 256;            // threads per block in every count kernel
constexpr int WAVES = WG / 64;

// ----------------------------------------------------------------------------
// small device helpers
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// position of the r-th set bit (r from 0) of w; w must have more than r bits set
__device__ __forceinline__ uint32_t select_bit(uint64_t w, uint32_t r) {
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
template <typename P>
__device__ __forceinline__ uint32_t seg_find(const P *seg, uint32_t d, uint32_t e) {
    uint32_t lo = 0, hi = d;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (seg[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// first j in [0, d) with nb[j] >= y, or d
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *nb, uint32_t d, uint32_t y) {
    uint32_t lo = 0, hi = d;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (nb[mid] < y) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t root_colour(uint64_t seed, uint32_t uid, uint32_t xid, uint32_t c) {
    return kc_colour(kc_mix64(seed ^ kc_mix64(((uint64_t)uid << 32) | xid)), c);
}
__device__ __forceinline__ uint32_t node_colour(uint64_t seed, uint32_t xid, uint32_t c) {
    return kc_colour(kc_mix64(seed ^ kc_mix64((uint64_t)xid)), c);
}

struct CountParams {
    const uint64_t *optr;
    const uint32_t *ocol;
    const uint32_t *rank2id;
    const uint32_t *queue;     // root ranks of this tier
    uint32_t count;            // roots in the queue
    uint32_t *next;            // dynamic queue cursor (zeroed before launch)
    uint64_t *per_root;        // optional, by original id
    unsigned long long *total; // global sum
    uint32_t *overflow;        // set when a sum does not fit in 64 bits
    int colored;
    int scheme;
    uint32_t c;
    uint64_t seed;
    // scratch tier
    uint64_t *gscratch;        // per-block slices
    size_t slice_words;        // u64 words per block slice
    uint32_t dcap;             // largest d the slice/LDS layout holds
};

__device__ __forceinline__ void add_total(const CountParams &p, uint64_t v, int ovf) {
    if (ovf) atomicOr(p.overflow, 1u);
    if (v == 0) return;
    const unsigned long long old = atomicAdd(p.total, (unsigned long long)v);
    if (old + v < old) atomicOr(p.overflow, 1u);
}

// ============================================================================
// Wave tier: d <= 64
// ============================================================================
template <int K>
struct WaveSmem {
    uint32_t nb[64];
    uint32_t seg[64];
    uint32_t epre[64];
    uint32_t colr[64];
    uint64_t delta[64];
    uint64_t rows[64];
    uint64_t stk[(K > 4 ? K - 4 : 1)][64];
    uint32_t task_next;
};

template <int K>
__global__ void __launch_bounds__(WG) k_count_wave(CountParams p) {
    __shared__ WaveSmem<K> sm_all[WAVES];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WaveSmem<K> &sm = sm_all[wave];
    constexpr int R = K - 3;  // nodes to choose below an edge task
    uint64_t wave_total = 0;
    int ovf = 0;

    for (;;) {
        uint32_t qi = 0;
        if (lane == 0) qi = atomicAdd(p.next, 1u);
        qi = __shfl(qi, 0, 64);
        if (qi >= p.count) break;
        const uint32_t u = p.queue[qi];
        const uint64_t base = p.optr[u];
        uint32_t d = (uint32_t)(p.optr[u + 1] - base);

        // Gamma+(u) into LDS; optionally cut to u's colour (global scheme)
        uint32_t a = lane < d ? p.ocol[base + lane] : 0xFFFFFFFFu;
        if (p.colored && p.scheme == KC_COLOR_GLOBAL) {
            const uint32_t cu = node_colour(p.seed, p.rank2id[u], p.c);
            const bool keep = lane < d && node_colour(p.seed, p.rank2id[a], p.c) == cu;
            const uint64_t bal = __ballot(keep);
            const uint32_t idx = (uint32_t)__popcll(bal & kc_lanemask_lt());
            sm.nb[lane] = 0xFFFFFFFFu;
            wave_sync();
            if (keep) sm.nb[idx] = a;
            wave_sync();
            d = (uint32_t)__popcll(bal);
            a = sm.nb[lane];
        }
        sm.nb[lane] = a;
        uint32_t len = 0;
        uint64_t ob = 0;
        if (lane < d) {
            ob = p.optr[a];
            len = (uint32_t)(p.optr[a + 1] - ob);
        }
        const uint32_t incl = kc_wave_incl_u32(len);
        const uint32_t excl = incl - len;
        const uint32_t Ttot = __shfl(incl, 63, 64);
        sm.seg[lane] = excl;
        sm.delta[lane] = ob - excl;
        sm.rows[lane] = 0;
        if (p.colored && p.scheme == KC_COLOR_PER_ROOT)
            sm.colr[lane] = lane < d ? root_colour(p.seed, p.rank2id[u], p.rank2id[a], p.c) : 0u;
        wave_sync();

        // staging: row i bit j = [a_j in Gamma+(a_i)]
        if (d > 0) {
            const uint32_t alast = sm.nb[d - 1];
            for (uint32_t e = lane; e < Ttot; e += 64) {
                const uint32_t i = seg_find(sm.seg, d, e);
                const uint32_t y = p.ocol[sm.delta[i] + e];
                if (y > alast) continue;
                const uint32_t j = lower_bound_u32(sm.nb, d, y);
                if (sm.nb[j] != y) continue;
                if (p.colored && p.scheme == KC_COLOR_PER_ROOT && sm.colr[i] != sm.colr[j]) continue;
                atomicOr((unsigned long long *)&sm.rows[i], 1ull << j);
            }
        }
        wave_sync();
        const uint64_t myrow = sm.rows[lane];

        uint64_t acc = 0;
        if constexpr (K == 3) {
            acc = (uint64_t)__popcll(myrow);
        } else {
            // edge tasks (i, j), j in row_i, enumerated through a prefix of row popcounts
            const uint32_t ce = (uint32_t)__popcll(myrow);
            const uint32_t ei = kc_wave_incl_u32(ce);
            const uint32_t E = __shfl(ei, 63, 64);
            sm.epre[lane] = ei - ce;
            if (lane == 0) sm.task_next = 0;
            wave_sync();
            int depth = -1;
            bool more = true;
            for (;;) {
                if (depth < 0 && more) {
                    const uint32_t t = atomicAdd(&sm.task_next, 1u);
                    if (t >= E) {
                        more = false;
                    } else {
                        const uint32_t i = seg_find(sm.epre, d, t);
                        const uint64_t ri = sm.rows[i];
                        const uint32_t j = select_bit(ri, t - sm.epre[i]);
                        const uint64_t P = ri & sm.rows[j];
                        if constexpr (R == 1) {
                            acc += (uint64_t)__popcll(P);
                        } else {
                            if ((uint32_t)__popcll(P) >= (uint32_t)R) {
                                depth = 0;
                                sm.stk[0][lane] = P;
                            }
                        }
                    }
                } else if (depth >= 0) {
                    if constexpr (R >= 2) {
                        uint64_t cur = sm.stk[depth][lane];
                        if (cur == 0) {
                            --depth;
                        } else {
                            const uint32_t v = (uint32_t)__builtin_ctzll(cur);
                            cur &= cur - 1;
                            sm.stk[depth][lane] = cur;
                            const uint64_t child = cur & sm.rows[v];
                            const int rem = R - depth - 1;  // nodes still to choose after v
                            if (rem == 1) {
                                acc += (uint64_t)__popcll(child);
                            } else if ((int)__popcll(child) >= rem) {
                                ++depth;
                                sm.stk[depth][lane] = child;
                            }
                        }
                    }
                }
                if (!__any(depth >= 0 || more)) break;
            }
        }
        const uint64_t q = kc_wave_sum_checked(acc, &ovf);
        if (lane == 0) {
            if (p.per_root) p.per_root[p.rank2id[u]] = q;
            const uint64_t nt = wave_total + q;
            if (nt < wave_total) ovf = 1;
            wave_total = nt;
        }
        wave_sync();
    }
    if (lane == 0) add_total(p, wave_total, ovf);
}

// ============================================================================
// Workgroup and scratch tiers: packed upper-triangular bitmap.
// Row i holds words (i+1)/64 .. W-1; its first word sits at
// rowoff(i) = i*W - sum_{t=1}^{i} floor(t/64).
// ============================================================================
__host__ __device__ inline uint64_t tri_rowoff(uint64_t i, uint64_t W) {
    const uint64_t q = i >> 6, r = i & 63;
    return i * W - (64 * (q * (q - (q ? 1 : 0)) / 2) + q * (r + 1));
}
__host__ __device__ inline uint64_t tri_words(uint64_t d) {
    const uint64_t W = (d + 63) / 64;
    return tri_rowoff(d, W);
}

// LDS / scratch layout of one workgroup for out-degree cap D and clique size k
struct WgLayout {
    size_t nb, seg, colr, delta, bm, stk, bytes;
    uint32_t W;
};
__host__ __device__ inline WgLayout wg_layout(uint32_t D, bool bitmap_inside) {
    WgLayout L;
    const uint32_t W = (D + 63) / 64;
    L.W = W;
    size_t o = 0;
    L.nb = o;    o += (size_t)D * 4;
    L.seg = o;   o += ((size_t)D + 1) * 4;
    L.colr = o;  o += (size_t)D * 4;
    o = (o + 7) & ~(size_t)7;
    L.delta = o; o += (size_t)D * 8;
    L.stk = o;   o += (size_t)WAVES * (KC_KMAX) * W * 8;
    L.bm = o;
    if (bitmap_inside) o += tri_words(D) * 8;
    L.bytes = o;
    return L;
}

template <bool GLOBAL>
__device__ __forceinline__ uint64_t *bm_row(uint64_t *bm, uint32_t i, uint32_t W) {
    return bm + tri_rowoff(i, W) - ((i + 1) >> 6);  // index with the absolute word number
}

template <int K, bool GLOBAL>
__global__ void __launch_bounds__(WG) k_count_wg(CountParams p) {
    extern __shared__ __align__(16) unsigned char smem_dyn[];
    __shared__ uint32_t s_misc[4];
    __shared__ uint64_t s_red[WAVES];
    __shared__ int s_ovf[WAVES];
    unsigned char *arena = GLOBAL ? (unsigned char *)(p.gscratch + (size_t)blockIdx.x * p.slice_words) : smem_dyn;
    const WgLayout L = wg_layout(p.dcap, true);
    uint32_t *nb = (uint32_t *)(arena + L.nb);
    uint32_t *seg = (uint32_t *)(arena + L.seg);
    uint32_t *colr = (uint32_t *)(arena + L.colr);
    uint64_t *delta = (uint64_t *)(arena + L.delta);
    uint64_t *stk_all = (uint64_t *)(arena + L.stk);
    uint64_t *bm = (uint64_t *)(arena + L.bm);
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t Wc = L.W;
    uint64_t *stk = stk_all + (size_t)wave * KC_KMAX * Wc;
    uint64_t block_total = 0;
    int ovf = 0;

    for (;;) {
        if (tid == 0) s_misc[0] = atomicAdd(p.next, 1u);
        __syncthreads();
        const uint32_t qi = s_misc[0];
        if (qi >= p.count) break;
        const uint32_t u = p.queue[qi];
        const uint64_t base = p.optr[u];
        uint32_t d = (uint32_t)(p.optr[u + 1] - base);

        for (uint32_t t = tid; t < d; t += WG) nb[t] = p.ocol[base + t];
        __syncthreads();
        if (p.colored && p.scheme == KC_COLOR_GLOBAL) {
            // keep only the nodes of u's colour, preserving order (block scan of flags)
            const uint32_t cu = node_colour(p.seed, p.rank2id[u], p.c);
            for (uint32_t t = tid; t < d; t += WG) seg[t] = node_colour(p.seed, p.rank2id[nb[t]], p.c) == cu ? 1u : 0u;
            __syncthreads();
            if (tid == 0) {
                uint32_t w = 0;
                for (uint32_t t = 0; t < d; ++t)
                    if (seg[t]) nb[w++] = nb[t];
                s_misc[1] = w;
            }
            __syncthreads();
            d = s_misc[1];
        }
        const uint32_t W = (d + 63) / 64;
        // out-degrees of Gamma+(u) and their exclusive prefix
        for (uint32_t t = tid; t < d; t += WG) {
            const uint32_t x = nb[t];
            seg[t] = (uint32_t)(p.optr[x + 1] - p.optr[x]);
            if (p.colored && p.scheme == KC_COLOR_PER_ROOT) colr[t] = root_colour(p.seed, p.rank2id[u], p.rank2id[x], p.c);
        }
        __syncthreads();
        if (tid < 64) {
            // one wave scans the d entries in chunks of 64
            uint32_t carry = 0;
            for (uint32_t c0 = 0; c0 < d; c0 += 64) {
                const uint32_t t = c0 + lane;
                const uint32_t v = t < d ? seg[t] : 0u;
                const uint32_t inc = kc_wave_incl_u32(v);
                if (t < d) {
                    seg[t] = carry + inc - v;
                    delta[t] = p.optr[nb[t]] - (carry + inc - v);
                }
                carry += __shfl(inc, 63, 64);
            }
            if (lane == 0) seg[d] = carry;
        }
        const uint64_t words = tri_words(d);
        for (uint64_t w = tid; w < words; w += WG) bm[w] = 0;
        __syncthreads();
        const uint32_t Ttot = seg[d];
        if (d > 0) {
            const uint32_t alast = nb[d - 1];
            for (uint32_t e = tid; e < Ttot; e += WG) {
                const uint32_t i = seg_find(seg, d, e);
                const uint32_t y = p.ocol[delta[i] + e];
                if (y > alast) continue;
                const uint32_t j = lower_bound_u32(nb, d, y);
                if (j >= d || nb[j] != y) continue;
                if (p.colored && p.scheme == KC_COLOR_PER_ROOT && colr[i] != colr[j]) continue;
                atomicOr((unsigned long long *)(bm_row<GLOBAL>(bm, i, W) + (j >> 6)), 1ull << (j & 63));
            }
        }
        if (tid == 0) s_misc[2] = 0;
        __syncthreads();

        // depth-first count, one first-level node per wave at a time
        uint64_t acc = 0;
        for (;;) {
            uint32_t i = 0;
            if (lane == 0) i = atomicAdd(&s_misc[2], 1u);
            i = __shfl(i, 0, 64);
            if (i >= d) break;
            const uint32_t lo0 = (i + 1) >> 6;
            const uint64_t *ri = bm_row<GLOBAL>(bm, i, W);
            if (K == 3) {
                for (uint32_t l = lo0 + lane; l < W; l += 64) acc += (uint64_t)__popcll(ri[l]);
                continue;
            }
            // stack[depth] holds the candidates not yet visited at that depth
            for (uint32_t l = lo0 + lane; l < W; l += 64) stk[l] = ri[l];
            uint32_t lo[KC_KMAX];
            lo[0] = lo0;
            int depth = 0;
            wave_sync();
            while (depth >= 0) {
                uint64_t *cur = stk + (size_t)depth * Wc;
                // lowest remaining candidate v at this depth
                int v = -1;
                for (uint32_t wb = lo[depth]; wb < W; wb += 64) {
                    const uint32_t l = wb + lane;
                    const uint64_t word = l < W ? cur[l] : 0ull;
                    const uint64_t bal = __ballot(word != 0);
                    if (bal) {
                        const uint32_t fl = (uint32_t)__builtin_ctzll(bal);
                        const uint64_t wsel = __shfl(word, fl, 64);
                        v = (int)((wb + fl) * 64 + (uint32_t)__builtin_ctzll(wsel));
                        if (lane == fl) cur[l] = word & (word - 1);
                        lo[depth] = wb + fl;
                        break;
                    }
                }
                wave_sync();
                if (v < 0) {
                    --depth;
                    continue;
                }
                const int rem = (K - 2) - depth - 1;  // nodes still to choose after v
                const uint32_t clo = ((uint32_t)v + 1) >> 6;
                const uint64_t *rv = bm_row<GLOBAL>(bm, (uint32_t)v, W);
                if (rem == 1) {
                    for (uint32_t l = clo + lane; l < W; l += 64) acc += (uint64_t)__popcll(cur[l] & rv[l]);
                } else {
                    uint64_t *nxt = cur + Wc;
                    uint32_t pc = 0;
                    for (uint32_t l = clo + lane; l < W; l += 64) {
                        const uint64_t x = cur[l] & rv[l];
                        nxt[l] = x;
                        pc += (uint32_t)__popcll(x);
                    }
                    pc = kc_wave_sum_u32(pc);
                    if ((int)pc >= rem) {
                        ++depth;
                        lo[depth] = clo;
                    }
                }
                wave_sync();
            }
        }
        // per-root total over the block
        int wovf = 0;
        const uint64_t wsum = kc_wave_sum_checked(acc, &wovf);
        if (lane == 0) {
            s_red[wave] = wsum;
            s_ovf[wave] = wovf;
        }
        __syncthreads();
        if (tid == 0) {
            uint64_t q = 0;
            for (int w = 0; w < WAVES; ++w) {
                const uint64_t nq = q + s_red[w];
                if (nq < q || s_ovf[w]) ovf = 1;
                q = nq;
            }
            if (p.per_root) p.per_root[p.rank2id[u]] = q;
            const uint64_t nt = block_total + q;
            if (nt < block_total) ovf = 1;
            block_total = nt;
        }
        __syncthreads();
    }
    if (tid == 0) add_total(p, block_total, ovf);
}

// ----------------------------------------------------------------------------
template <int K>
void launch_tiers(const CountParams &base, const kc_queue &q, uint32_t *cursors, int cus, size_t lds_max,
                  hipStream_t s, uint64_t *gscratch, size_t slice_words, uint32_t scratch_blocks) {
    const uint32_t *queue = q.buf.as<uint32_t>();
    // scratch tier first: the largest roots
    if (q.count[2]) {
        CountParams p = base;
        p.queue = queue + q.offset[2];
        p.count = q.count[2];
        p.next = cursors + 2;
        p.gscratch = gscratch;
        p.slice_words = slice_words;
        p.dcap = q.max_d[2];
        hipLaunchKernelGGL((k_count_wg<K, true>), dim3(scratch_blocks), dim3(WG), 0, s, p);
    }
    if (q.count[1]) {
        CountParams p = base;
        p.queue = queue + q.offset[1];
        p.count = q.count[1];
        p.next = cursors + 1;
        p.dcap = q.max_d[1] < 65 ? 65 : q.max_d[1];
        const WgLayout L = wg_layout(p.dcap, true);
        const uint32_t per_cu = (uint32_t)(lds_max / (L.bytes + 1024));
        uint32_t blocks = (uint32_t)cus * (per_cu ? per_cu : 1);
        if (blocks > q.count[1]) blocks = q.count[1];
        (void)hipFuncSetAttribute((const void *)&k_count_wg<K, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)L.bytes);
        hipLaunchKernelGGL((k_count_wg<K, false>), dim3(blocks), dim3(WG), L.bytes, s, p);
    }
    if (q.count[0]) {
        CountParams p = base;
        p.queue = queue + q.offset[0];
        p.count = q.count[0];
        p.next = cursors + 0;
        uint32_t blocks = (q.count[0] + WAVES - 1) / WAVES;
        const uint32_t cap = (uint32_t)cus * 8;
        if (blocks > cap) blocks = cap;
        hipLaunchKernelGGL((k_count_wave<K>), dim3(blocks), dim3(WG), 0, s, p);
    }
}

struct DevInfo {
    int cus = 0;
    size_t lds_max = 0;
};
DevInfo dev_info(int device) {
    static DevInfo cache[64];
    static int have[64] = {0};
    if (device >= 0 && device < 64 && have[device]) return cache[device];
    DevInfo di;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess) di.cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess)
        di.lds_max = (size_t)v;
    if (di.cus <= 0) di.cus = 256;
    if (di.lds_max == 0) di.lds_max = 65536;
    if (device >= 0 && device < 64) {
        cache[device] = di;
        have[device] = 1;
    }
    return di;
}

}  // namespace

// Largest out-degree whose workgroup layout (packed bitmap included) fits in LDS.
uint32_t kc_lds_dcap(int device) {
    const DevInfo di = dev_info(device);
    const size_t budget = di.lds_max - 2048;  // static shared arrays of the kernel
    uint32_t lo = 64, hi = 1 << 16;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        if (wg_layout(mid, true).bytes <= budget) lo = mid; else hi = mid - 1;
    }
    return lo;
}

size_t kc_scratch_slice_words(uint32_t dmax) {
    return (wg_layout(dmax, true).bytes + 7) / 8;
}

kc_status kc_count_impl(const kc_graph *g, const kc_count_args &a, uint64_t *total, int *overflow) {
    hipStream_t s = g->stream;
    const DevInfo di = dev_info(g->device);
    const uint32_t dcap = kc_lds_dcap(g->device);

    KC_HIP(hipEventRecord(g->ev[0], s));
    kc_queue q;
    KC_TRY(kc_build_queue(g, a.k, a.policy, dcap, q));
    KC_HIP(hipEventRecord(g->ev[1], s));

    // device result area: [0] total, [1] overflow, [2..5] tier cursors
    KC_HIP(hipMemsetAsync(g->d_res, 0, 8 * sizeof(uint64_t), s));
    const char *bias = getenv("KC_TEST_TOTAL_BIAS");  // test hook: forces the overflow path
    if (bias) {
        const unsigned long long b = strtoull(bias, nullptr, 0);
        KC_HIP(hipMemcpyAsync(g->d_res, &b, sizeof(b), hipMemcpyHostToDevice, s));
    }
    CountParams p{};
    p.optr = g->optr;
    p.ocol = g->ocol;
    p.rank2id = g->rank2id;
    p.per_root = a.per_root;
    p.total = (unsigned long long *)g->d_res;
    p.overflow = (uint32_t *)(g->d_res + 1);
    p.colored = a.colored;
    p.scheme = a.scheme;
    p.c = a.c;
    p.seed = a.seed;
    uint32_t *cursors = (uint32_t *)(g->d_res + 2);

    if (a.per_root) KC_HIP(hipMemsetAsync(a.per_root, 0, (size_t)g->n * sizeof(uint64_t), s));

    kc_tmp gscr;
    size_t slice_words = 0;
    uint32_t scratch_blocks = 0;
    if (q.count[2]) {
        slice_words = kc_scratch_slice_words(q.max_d[2]);
        scratch_blocks = q.count[2] < (uint32_t)di.cus ? q.count[2] : (uint32_t)di.cus;
        // bound the scratch footprint to 8 GiB
        while (scratch_blocks > 1 && slice_words * 8 * scratch_blocks > (8ull << 30)) scratch_blocks /= 2;
        KC_TRY(kc_tmp_alloc(gscr, slice_words * 8 * scratch_blocks, s));
    }
    switch (a.k) {
#define KC_CASE(KK)                                                                                           \
    case KK:                                                                                                  \
        launch_tiers<KK>(p, q, cursors, di.cus, di.lds_max, s, gscr.as<uint64_t>(), slice_words, scratch_blocks); \
        break;
        KC_CASE(3)
        KC_CASE(4)
        KC_CASE(5)
        KC_CASE(6)
        KC_CASE(7)
        KC_CASE(8)
        KC_CASE(9)
        KC_CASE(10)
#undef KC_CASE
        default:
            return kc_fail(KC_EINVAL, "k=%d outside the counting kernels' range", a.k);
    }
    KC_HIP(hipGetLastError());
    KC_HIP(hipEventRecord(g->ev[2], s));
    KC_HIP(hipMemcpyAsync(g->h_res, g->d_res, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    KC_HIP(hipStreamSynchronize(s));
    float t_sched = 0.f, t_count = 0.f;
    (void)hipEventElapsedTime(&t_sched, g->ev[0], g->ev[1]);
    (void)hipEventElapsedTime(&t_count, g->ev[1], g->ev[2]);
    kc_graph *gm = const_cast<kc_graph *>(g);
    gm->t_schedule = t_sched;
    gm->t_count = t_count;
    gm->t_total = t_sched + t_count;
    *total = g->h_res[0];
    *overflow = g->h_res[1] != 0;
    return KC_OK;
}
