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
//   wave       d <= 64: one wave per root; G+(u) is a local graph of one 64-bit
//              row per node, counted by the lane state machine below.
//   workgroup  64 < d <= D_LDS: one workgroup per root, packed upper-triangular
//              bitmap in LDS.  Waves take first-level nodes v; a candidate set
//              of at most 64 (128) nodes is compacted into a one-word (two-word)
//              local graph and counted by the lane state machine, larger ones
//              are split one level further.
//   scratch    d > D_LDS: as workgroup, bitmap in a global-memory slice.
// Every count is an exact uint64; sums are carry-checked.
#include "kc_internal.h"

namespace {

constexpr int WG = 256;  // threads per block in every count kernel
constexpr int WAVES = WG / 64;

// ----------------------------------------------------------------------------
// small device helpers (wave sync, bit select, segment search: kc_internal.h)
// first j in [0, d) with nb[j] >= y, or d
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *nb, uint32_t d, uint32_t y) {
    uint32_t lo = 0, hi = d;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (nb[mid] < y) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Open-addressing table (LDS) from a node's rank to its position in Gamma+(u):
// 16-bit slots hold positions (0xFFFF = empty), verified against nb[]; a slot
// is claimed by a compare-and-swap on the 32-bit word that contains it.
constexpr uint32_t HEMPTY = 0xFFFFFFFFu;
__host__ __device__ inline uint32_t hash_bits(uint32_t D) {
    uint32_t b = 6;
    while ((1u << b) < 2 * D) ++b;
    return b;
}
__device__ __forceinline__ uint32_t hash_slot(uint32_t y, uint32_t bits) { return (y * 2654435769u) >> (32 - bits); }
__device__ __forceinline__ void hash_insert(uint16_t *tab, uint32_t bits, uint32_t y, uint32_t pos) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t h = hash_slot(y, bits);
    uint32_t *words = reinterpret_cast<uint32_t *>(tab);
    for (;;) {
        uint32_t *w = &words[h >> 1];
        const uint32_t sh = (h & 1u) * 16u;
        uint32_t old = *w;
        bool done = false;
        while (((old >> sh) & 0xFFFFu) == 0xFFFFu) {
            const uint32_t upd = (old & ~(0xFFFFu << sh)) | (pos << sh);
            const uint32_t seen = atomicCAS(w, old, upd);
            if (seen == old) {
                done = true;
                break;
            }
            old = seen;
        }
        if (done) return;
        h = (h + 1) & mask;
    }
}
// position of y among nb[0, d), or HEMPTY
__device__ __forceinline__ uint32_t hash_find(const uint16_t *tab, uint32_t bits, const uint32_t *nb, uint32_t y) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t h = hash_slot(y, bits);
    for (;;) {
        const uint32_t j = tab[h];
        if (j == 0xFFFFu) return HEMPTY;
        if (nb[j] == y) return j;
        h = (h + 1) & mask;
    }
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
    const uint32_t *queue;      // root ranks of this tier
    uint32_t count;             // roots in the queue
    uint32_t *next;             // dynamic queue cursor (zeroed before launch)
    uint64_t *per_root;         // optional, by original id
    unsigned long long *total;  // global sum
    uint32_t *overflow;         // set when a sum does not fit in 64 bits
    int colored;
    int scheme;
    uint32_t c;
    uint64_t seed;
    uint64_t *gscratch;   // scratch tier: per-block slices
    size_t slice_words;   // u64 words per slice
    uint32_t dcap;        // largest d the workgroup layout holds
    uint32_t chunk_div;   // queue chunk = count / (workers * chunk_div)
    uint32_t local2;      // workgroup tier, k >= 6: compact candidate sets of 65..128 nodes into two-word local graphs
    // workgroup tier, split roots: item = rank << 32 | part << 16 | parts (null: queue, one part each)
    const uint64_t *items;
    // batches: graph of every rank and one total per graph (null for one graph)
    const uint32_t *graph_of;
    unsigned long long *gtotals;
    // staged G+(u) cache of the handle: wave-tier rows, larger roots' bitmaps
    uint64_t *lrows;
    uint64_t *wbits;
    uint32_t stage_wd;          // roots of out-degree <= stage_wd keep rows at lrows, larger ones bitmaps
    const uint64_t *wbits_raw;  // the staged bitmaps as staged (before any pair-sampling mask)
    uint32_t *wedges;           // staging: edges of each workgroup-tier G+(u), by rank (optional)
    unsigned long long *slots;  // 32 partial totals of a single-graph count (summed into *total)
    const uint64_t *woff;
};


// Queue counters: chunk c of a queue is handed out by counter c mod QCTR, the
// counters QCTR_STRIDE u32 (256 bytes) apart so that their atomics do not
// serialise on one address; beside each (QCTR_FLAG u32 further, on another cache
// line) a flag is set once the counter is spent.
constexpr uint32_t QCTR = 32;
constexpr uint32_t QCTR_STRIDE = 64;
constexpr uint32_t QCTR_FLAG = 32;

// Next chunk start of a queue for the calling wave (all 64 lanes call it), or
// 0xFFFFFFFF once every counter is spent.  The wave starts at its home counter;
// `dead` holds the counters it has seen spent.  Once the home counter is spent,
// the others are first read (flags and values, one lane each, past the compute
// unit's cache) and only a live one is taken with an atomic: at the end of a
// queue the whole grid looks for work at once, and device-scope atomics on a
// few addresses serialise.  Each pass either returns or adds a counter to
// `dead`, so it ends within QCTR passes.
__device__ __forceinline__ uint32_t next_chunk(uint32_t *ctr, uint32_t count, uint32_t chunk, uint32_t home,
                                               uint32_t &dead) {
    const uint32_t lane = kc_lane();
    uint32_t x = home;
    for (;;) {
        if (!((dead >> x) & 1u)) {
            uint32_t b = 0xFFFFFFFFu;
            if (lane == 0) {
                const uint64_t c = (uint64_t)atomicAdd(ctr + x * QCTR_STRIDE, 1u) * QCTR + x;
                if (c * chunk < count) b = (uint32_t)(c * chunk);
                else __hip_atomic_store(ctr + x * QCTR_STRIDE + QCTR_FLAG, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            b = __shfl(b, 0, 64);
            if (b != 0xFFFFFFFFu) return b;
            dead |= 1u << x;
        }
        bool live = false;
        if (lane < QCTR && !((dead >> lane) & 1u)) {
            const uint32_t f = __hip_atomic_load(ctr + lane * QCTR_STRIDE + QCTR_FLAG, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t v = __hip_atomic_load(ctr + lane * QCTR_STRIDE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            live = f == 0u && ((uint64_t)v * QCTR + lane) * chunk < count;  // counters only grow
        }
        const uint64_t lm = __ballot(live);
        dead |= ~(uint32_t)lm;  // a counter seen spent stays spent
        if (!lm) return 0xFFFFFFFFu;
        const uint64_t after = lm & ~((2ull << x) - 1ull);  // live counters past x
        x = (uint32_t)__builtin_ctzll(after ? after : lm);
    }
}

// Roots per queue fetch: one device-scope atomic serves a chunk of roots.
__device__ __forceinline__ uint32_t queue_chunk(uint32_t count, uint32_t workers, uint32_t div) {
    const uint32_t c = count / (workers * div);
    return c < 1u ? 1u : (c > 64u ? 64u : c);
}

// add a (graph's) partial sum to its total, carry-checked.  A single graph's total
// is spread over 32 slots (by the caller's `spread`, e.g. its block), summed by
// k_total_slots: device-scope atomics on one address serialise when the whole
// grid finishes at once.
__device__ __forceinline__ void add_to(const CountParams &p, uint32_t gid, uint64_t v, int ovf, uint32_t spread = 0) {
    if (ovf) atomicOr(p.overflow, 1u);
    if (v == 0) return;
    unsigned long long *dst = p.gtotals ? p.gtotals + gid : p.slots + (spread & 31u);
    const unsigned long long old = atomicAdd(dst, (unsigned long long)v);
    if (old + v < old) atomicOr(p.overflow, 1u);
}

// ============================================================================
// Local graphs of at most 64 nodes: one 64-bit upper-triangular row per node.
// local_count adds the number of ell-cliques of such a graph to the lanes' acc.
// For ell >= 3 the cliques are enumerated below the edges (i, j) of the local
// graph: every lane runs its own depth-first state machine over one edge's
// candidate set P = row_i & row_j and takes a new edge when it is done, so lanes
// do not wait for each other's subtrees.
// Rows of lanes >= s must be zero.
// ============================================================================
// NS = depth-first stack entries: counting ell-cliques uses ell - 3 of them, or
// ell - 4 when a node that needs two more nodes counts the edges inside its
// candidate set in place (INPLACE2 below); at least one.
// Depth-first stack levels kept in registers; deeper stacks live in LDS (where
// registers would spill).  The one-wave kernel keeps two levels, the
// workgroup kernel two as well (three spill).
constexpr int LC_LDS_FROM = 2;  // local areas hold LDS stacks for more levels than this
constexpr int LC_REG_WAVE = 2;
constexpr int LC_REG_WG = 2;
// Edges of a local graph listed in LDS (i << 8 | j) when there are at most this many;
// a task is then one read instead of a segment search and a bit selection.
constexpr uint32_t LC_ELIST = 512;

template <int NS>
struct LocalArea {
    uint64_t rows[64];
    uint32_t epre[64];
    union {
        uint32_t members[64];       // compaction (before counting)
        uint16_t elist[LC_ELIST];   // counting
    };
    uint64_t stk[NS > LC_LDS_FROM ? NS : 0][64];  // depth-first stacks when too deep for registers
};

// Per-lane depth-first stacks of at most N levels live in registers: an entry
// is read or written through a chain of selects on the depth.
template <int N>
__device__ __forceinline__ uint64_t st_get(const uint64_t (&st)[N], int d) {
    uint64_t v = st[0];
#pragma unroll
    for (int i = 1; i < N; ++i) v = d == i ? st[i] : v;
    return v;
}
template <int N>
__device__ __forceinline__ void st_set(uint64_t (&st)[N], int d, uint64_t v) {
#pragma unroll
    for (int i = 0; i < N; ++i) st[i] = d == i ? v : st[i];
}

// SPREAD3: unlisted edges at R = 3 (below) are also shared out a fixed set per
// lane rather than through the state machine.
// Edges inside the node set P of a one-word local graph: sum over v in P of
// |P_{>v} & row_v|.  Four members per step, so that four row reads are in flight
// at once (a member past the end reads row 0 and adds nothing: its remainder is 0).
__device__ __forceinline__ uint32_t edges_inside(uint64_t P, const uint64_t *rows) {
    uint32_t c = 0;
    while (P) {
        const uint32_t v0 = (uint32_t)__builtin_ctzll(P);
        P &= P - 1;
        const uint64_t P1 = P;
        const uint32_t v1 = P ? (uint32_t)__builtin_ctzll(P) : 0u;
        P &= P - 1;
        const uint64_t P2 = P;
        const uint32_t v2 = P ? (uint32_t)__builtin_ctzll(P) : 0u;
        P &= P - 1;
        const uint64_t P3 = P;
        const uint32_t v3 = P ? (uint32_t)__builtin_ctzll(P) : 0u;
        P &= P - 1;
        const uint64_t r0 = rows[v0], r1 = rows[v1], r2 = rows[v2], r3 = rows[v3];
        c += (uint32_t)(__popcll(P1 & r0) + __popcll(P2 & r1) + __popcll(P3 & r2) + __popcll(P & r3));
    }
    return c;
}

// INPLACE2: a node that needs two more nodes counts the edges inside its candidate
// set in place (one-wave tier: small, sparse local graphs, where this saves most of
// the state machine's steps); otherwise it is pushed and its members are taken one
// step each (workgroup tier: dense candidate sets, where the in-place loops leave
// the other lanes idle).
// First-node filter (fpart, fparts): only the cliques whose first (lowest) node has a
// local index congruent to fpart modulo fparts are counted; (0, 1) counts all.  The
// split items of the heaviest nodes (Section 7) share a node's subtree this way.
template <int REGL, bool SPREAD3, bool INPLACE2, int NS>
__device__ __forceinline__ void local_count(LocalArea<NS> &A, uint32_t s, int ell, uint64_t &acc,
                                            uint32_t fpart = 0, uint32_t fparts = 1) {
    static_assert(REGL >= LC_LDS_FROM, "levels neither in registers nor in LDS");
    const uint32_t lane = kc_lane();
    const uint64_t row = A.rows[lane];
    const bool mine = fparts == 1 || lane % fparts == fpart;  // this lane's row may start cliques
    if (ell <= 1) {
        if (lane == 0) acc += ell == 1 ? (fparts == 1 ? s : (s > fpart ? (s - fpart + fparts - 1) / fparts : 0u)) : 1u;
        return;
    }
    if (ell == 2) {
        if (mine) acc += (uint64_t)__popcll(row);
        return;
    }
    const int R = ell - 2;  // nodes to choose inside an edge's candidate set
    const uint32_t ce = mine ? (uint32_t)__popcll(row) : 0u;
    const uint32_t ei = kc_wave_incl_u32(ce);
    const uint32_t E = __shfl(ei, 63, 64);
    const bool listed = E <= LC_ELIST;
    if (listed) {
        uint64_t r = mine ? row : 0ull;
        uint32_t pos = ei - ce;
        while (r) {
            A.elist[pos++] = (uint16_t)((lane << 8) | (uint32_t)__builtin_ctzll(r));
            r &= r - 1;
        }
    } else {
        A.epre[lane] = ei - ce;
    }
    kc_wave_sync();
    if (R <= 2 || (R == 3 && (listed || SPREAD3))) {
        // Up to three levels below an edge: lane l takes edges l, l + 64, ...  An
        // edge task (i, j) adds the (R+1)-cliques of the candidate set
        // P = row_i & row_j: its size (R = 1), one intersection per member (R = 2),
        // one per edge inside it (R = 3).  The edge is read from the list, or
        // found from the row starts: lane r holds row r's first edge, and the
        // rows starting in a batch of 64 edges are scanned once by the whole wave.
        // Unlisted edges at R = 3 go to the state machine below unless SPREAD3:
        // their subtrees can vary too much for a fixed share per lane (dense
        // candidate sets in the workgroup tier), while the one-wave tier's small
        // roots gain from the simpler loop.
        const uint32_t start = ei - ce;
        uint32_t r0 = 0;  // the row holding the batch's first edge
        for (uint32_t b = 0; b < E; b += 64) {
            const uint32_t t = b + lane;
            uint64_t P;
            if (listed) {
                const uint32_t e = t < E ? A.elist[t] : 0u;
                P = t < E ? A.rows[e >> 8] & A.rows[e & 255u] : 0ull;
            } else {
                uint32_t i = r0;
                for (uint32_t x = r0 + 1; x < s; ++x) {
                    const uint32_t sx = (uint32_t)__builtin_amdgcn_readlane((int)start, (int)x);
                    if (sx >= b + 64) break;
                    if (sx <= t) i = x;
                }
                r0 = (uint32_t)__builtin_amdgcn_readlane((int)i, 63);
                const uint64_t ri = A.rows[i];
                P = t < E ? ri & A.rows[kc_select_bit(ri, t - A.epre[i])] : 0ull;
            }
            if (R == 1) {
                acc += (uint64_t)__popcll(P);
            } else if (R == 2) {
                acc += edges_inside(P, A.rows);
            } else {
                // four members per step as in edges_inside: their row reads in flight together
                while (P) {
                    const uint32_t v0 = (uint32_t)__builtin_ctzll(P);
                    P &= P - 1;
                    const uint64_t P1 = P;
                    const uint32_t v1 = P ? (uint32_t)__builtin_ctzll(P) : 0u;
                    P &= P - 1;
                    const uint64_t P2 = P;
                    const uint32_t v2 = P ? (uint32_t)__builtin_ctzll(P) : 0u;
                    P &= P - 1;
                    const uint64_t P3 = P;
                    const uint32_t v3 = P ? (uint32_t)__builtin_ctzll(P) : 0u;
                    P &= P - 1;
                    const uint64_t r0 = A.rows[v0], r1 = A.rows[v1], r2 = A.rows[v2], r3 = A.rows[v3];
                    acc += edges_inside(P1 & r0, A.rows) + edges_inside(P2 & r1, A.rows) +
                           edges_inside(P3 & r2, A.rows) + edges_inside(P & r3, A.rows);
                }
            }
        }
        kc_wave_sync();
        return;
    }
    // Idle lanes are refilled together, once at least REFILL of them wait (or
    // no lane is busy): task t of the i-th idle lane is next + i.
    constexpr uint32_t REFILL = 16;
    constexpr bool REG = NS <= REGL;
    uint64_t st[REG ? NS : 1];
#pragma unroll
    for (int l = 0; l < (REG ? NS : 1); ++l) st[l] = 0;
    auto sget = [&](int dd) -> uint64_t {
        if constexpr (REG) return st_get(st, dd);
        else return A.stk[dd][lane];
    };
    auto sset = [&](int dd, uint64_t v) {
        if constexpr (REG) st_set(st, dd, v);
        else A.stk[dd][lane] = v;
    };
    int depth = -1;
    uint32_t next = 0;
    for (;;) {
        const uint64_t idle = __ballot(depth < 0);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (next < E && (nidle >= REFILL || nidle == 64)) {
            const uint32_t t = next + (uint32_t)__popcll(idle & kc_lanemask_lt());
            next += nidle;
            if (depth < 0 && t < E) {
                uint64_t P;
                if (listed) {
                    const uint32_t e = A.elist[t];
                    P = A.rows[e >> 8] & A.rows[e & 255u];
                } else {
                    const uint32_t i = kc_seg_find(A.epre, s, t);
                    const uint64_t ri = A.rows[i];
                    P = ri & A.rows[kc_select_bit(ri, t - A.epre[i])];
                }
                if (R == 1) {
                    acc += (uint64_t)__popcll(P);
                } else if ((int)__popcll(P) >= R) {
                    depth = 0;
                    sset(0, P);
                }
            }
        } else if (nidle == 64) {
            break;
        }
        if (depth >= 0) {
            uint64_t cur = sget(depth);
            const int rem = R - depth - 1;  // nodes still to choose after the next member
            if (cur == 0) {
                --depth;
            } else {
                const uint32_t v = (uint32_t)__builtin_ctzll(cur);
                cur &= cur - 1;
                sset(depth, cur);
                const uint64_t child = cur & A.rows[v];
                if (rem == 1) {
                    acc += (uint64_t)__popcll(child);
                } else if (INPLACE2 && rem == 2) {
                    // the edges inside the child set, four members per step, in place
                    acc += edges_inside(child, A.rows);
                } else if ((int)__popcll(child) >= rem) {
                    ++depth;
                    sset(depth, child);
                }
            }
        }
    }
    kc_wave_sync();
}

// ============================================================================
// Two-word local graphs: at most 128 nodes, row t held in rows[t][0..1].  The
// same edge-task state machine as local_count, with two-word candidate sets.
// Rows t >= s must be zero.
// ============================================================================
template <int NS>
struct LocalArea2 {
    uint64_t rows[128][2];
    uint32_t epre[128];
    uint32_t members[128];
    uint64_t stk[NS > LC_LDS_FROM ? NS : 0][2][64];  // depth-first stacks when too deep for registers
};

__device__ __forceinline__ uint32_t select_bit2(uint64_t w0, uint64_t w1, uint32_t r) {
    const uint32_t c0 = (uint32_t)__popcll(w0);
    return r < c0 ? kc_select_bit(w0, r) : 64u + kc_select_bit(w1, r - c0);
}

// (fpart, fparts): the first-node filter of local_count.
template <int NS>
__device__ __forceinline__ void local_count2(LocalArea2<NS> &A, uint32_t s, int ell, uint64_t &acc,
                                             uint32_t fpart = 0, uint32_t fparts = 1) {
    const uint32_t lane = kc_lane();
    // this lane's two rows 2*lane and 2*lane+1 (consecutive, so the task prefix stays ordered)
    const bool ma = fparts == 1 || (2 * lane) % fparts == fpart, mb = fparts == 1 || (2 * lane + 1) % fparts == fpart;
    const uint32_t ca = ma ? (uint32_t)(__popcll(A.rows[2 * lane][0]) + __popcll(A.rows[2 * lane][1])) : 0u;
    const uint32_t cb = mb ? (uint32_t)(__popcll(A.rows[2 * lane + 1][0]) + __popcll(A.rows[2 * lane + 1][1])) : 0u;
    if (ell <= 1) {
        if (lane == 0) acc += ell == 1 ? (fparts == 1 ? s : (s > fpart ? (s - fpart + fparts - 1) / fparts : 0u)) : 1u;
        return;
    }
    if (ell == 2) {
        acc += ca + cb;
        return;
    }
    const int R = ell - 2;
    const uint32_t incl = kc_wave_incl_u32(ca + cb);
    const uint32_t E = __shfl(incl, 63, 64);
    const uint32_t sa = incl - ca - cb, sb = incl - cb;  // first edges of rows 2*lane, 2*lane+1
    A.epre[2 * lane] = sa;
    A.epre[2 * lane + 1] = sb;
    kc_wave_sync();
    if (R <= 2) {
        // as in local_count: lane l takes edges l, l + 64, ..., each edge's row
        // found from the row starts that fall in its batch of 64 edges
        uint32_t r0 = 0;
        for (uint32_t b = 0; b < E; b += 64) {
            const uint32_t t = b + lane;
            uint32_t i = r0;
            for (uint32_t x = r0 + 1; x < s; ++x) {
                const uint32_t sx = (uint32_t)__builtin_amdgcn_readlane((int)((x & 1u) ? sb : sa), (int)(x >> 1));
                if (sx >= b + 64) break;
                if (sx <= t) i = x;
            }
            r0 = (uint32_t)__builtin_amdgcn_readlane((int)i, 63);
            uint64_t p0 = 0, p1 = 0;
            if (t < E) {
                const uint64_t r0w = A.rows[i][0], r1w = A.rows[i][1];
                const uint32_t j = select_bit2(r0w, r1w, t - A.epre[i]);
                p0 = r0w & A.rows[j][0];
                p1 = r1w & A.rows[j][1];
            }
            if (R == 1) {
                acc += (uint64_t)(__popcll(p0) + __popcll(p1));
                continue;
            }
            while (p0 | p1) {
                uint32_t v;
                if (p0) {
                    v = (uint32_t)__builtin_ctzll(p0);
                    p0 &= p0 - 1;
                } else {
                    v = 64u + (uint32_t)__builtin_ctzll(p1);
                    p1 &= p1 - 1;
                }
                acc += (uint64_t)(__popcll(p0 & A.rows[v][0]) + __popcll(p1 & A.rows[v][1]));
            }
        }
        kc_wave_sync();
        return;
    }
    constexpr uint32_t REFILL = 16;
    constexpr bool REG = NS <= LC_LDS_FROM;
    uint64_t st0[REG ? NS : 1], st1[REG ? NS : 1];
#pragma unroll
    for (int l = 0; l < (REG ? NS : 1); ++l) st0[l] = st1[l] = 0;
    auto sget = [&](int dd, uint64_t &a0, uint64_t &a1) {
        if constexpr (REG) {
            a0 = st_get(st0, dd);
            a1 = st_get(st1, dd);
        } else {
            a0 = A.stk[dd][0][lane];
            a1 = A.stk[dd][1][lane];
        }
    };
    auto sset = [&](int dd, uint64_t v0, uint64_t v1) {
        if constexpr (REG) {
            st_set(st0, dd, v0);
            st_set(st1, dd, v1);
        } else {
            A.stk[dd][0][lane] = v0;
            A.stk[dd][1][lane] = v1;
        }
    };
    int depth = -1;
    uint32_t next = 0;
    for (;;) {
        const uint64_t idle = __ballot(depth < 0);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (next < E && (nidle >= REFILL || nidle == 64)) {
            const uint32_t t = next + (uint32_t)__popcll(idle & kc_lanemask_lt());
            next += nidle;
            if (depth < 0 && t < E) {
                const uint32_t i = kc_seg_find(A.epre, s, t);
                const uint64_t r0 = A.rows[i][0], r1 = A.rows[i][1];
                const uint32_t j = select_bit2(r0, r1, t - A.epre[i]);
                const uint64_t p0 = r0 & A.rows[j][0], p1 = r1 & A.rows[j][1];
                const int pc = __popcll(p0) + __popcll(p1);
                if (R == 1) {
                    acc += (uint64_t)pc;
                } else if (pc >= R) {
                    depth = 0;
                    sset(0, p0, p1);
                }
            }
        } else if (nidle == 64) {
            break;
        }
        if (depth >= 0) {
            uint64_t c0, c1;
            sget(depth, c0, c1);
            if ((c0 | c1) == 0) {
                --depth;
            } else {
                uint32_t v;
                if (c0) {
                    v = (uint32_t)__builtin_ctzll(c0);
                    c0 &= c0 - 1;
                } else {
                    v = 64u + (uint32_t)__builtin_ctzll(c1);
                    c1 &= c1 - 1;
                }
                sset(depth, c0, c1);
                const uint64_t h0 = c0 & A.rows[v][0], h1 = c1 & A.rows[v][1];
                const int pc = __popcll(h0) + __popcll(h1);
                const int rem = R - depth - 1;
                if (rem == 1) {
                    acc += (uint64_t)pc;
                } else if (pc >= rem) {
                    ++depth;
                    sset(depth, h0, h1);
                }
            }
        }
    }
    kc_wave_sync();
}

// ============================================================================
// Wave tier: d <= 64.  Consecutive roots of the queue whose out-degrees sum to
// at most 64 share one wave pass: their G+(u) are laid side by side as the
// diagonal blocks of one 64-node local graph (no edge joins two blocks, so its
// cliques are exactly the union of the roots' cliques).  When per-root counts
// are requested, or with the global colouring (which cuts Gamma+(u) first),
// every pass holds one root.
// ============================================================================
// Kernel modes: stage G+(u) and count it; stage it into the handle's cache
// only; count from the cache.
constexpr int MODE_STAGE = 0;
constexpr int MODE_STORE = 1;
constexpr int MODE_CACHED = 2;

// 64-element windows of flattened out-lists read per staging step
constexpr uint32_t STAGE_WINDOWS = 4;

// Staging state of one wave pass, overlaid on the local-graph area (whose
// rows it shares; the rest of that area is idle until counting starts).
struct WaveStage {
    uint64_t rows[64];
    uint32_t filt[64];  // 2048-bit membership filter of the packed Gamma+ lists
    uint32_t qy[128];   // ring of filter survivors: out-list element ...
    uint8_t qi[128];    // ... and the list (local node) it came from
    uint8_t flag[64 * STAGE_WINDOWS];  // per step: 1 + the list starting at each slot
};
static_assert(offsetof(WaveStage, rows) == 0 && offsetof(LocalArea<1>, rows) == 0,
              "staging rows must alias the local graph's rows");

// The one-wave tier counts in place from k = 8 on (planted 4M, k = 8: 169 ms to 97 ms
// with the tier's base chunk size); at k = 7 it made no measurable difference.
constexpr bool wave_inplace(int k) { return k >= 8; }
constexpr int wave_stack(int k) {
    return wave_inplace(k) ? (k - 5 > 1 ? k - 5 : 1) : (k - 4 > 1 ? k - 4 : 1);
}

template <int K>
struct WaveSmem {
    union {
        LocalArea<wave_stack(K)> A;
        WaveStage S;
    };
    uint32_t nb[64];      // the packed Gamma+ lists
    uint32_t colr[64];
    uint32_t rstart[64];  // first lane of each packed root
    uint8_t blo[64], bhi[64];  // block [blo, bhi) of each lane
    uint64_t delta[64];   // out-list base minus its first flattened element
};

__device__ __forceinline__ uint32_t filt_hash(uint32_t y) { return (y * 2654435769u) >> 21; }

// Exact test of cnt (<= 64) filter survivors from the ring at qh: set bit j of
// row i when the element y of a_i's out-list is a_j of i's own block.
template <int K>
__device__ __forceinline__ void wave_stage_check(WaveSmem<K> &sm, uint32_t qh, uint32_t cnt, bool percol) {
    const uint32_t lane = kc_lane();
    if (lane < cnt) {
        const uint32_t slot = (qh + lane) & 127u;
        const uint32_t y = sm.S.qy[slot], i = sm.S.qi[slot];
        const uint32_t lo = sm.blo[i], hi = sm.bhi[i];
        const uint32_t j = lo + lower_bound_u32(sm.nb + lo, hi - lo, y);
        if (j < hi && sm.nb[j] == y && (!percol || sm.colr[i] == sm.colr[j]))
            atomicOr((unsigned long long *)&sm.A.rows[i], 1ull << j);
    }
}

// Register target of the one-wave kernel: eight waves per SIMD from k = 7 (a few
// spilled registers; planted 4M one-wave tier k = 7 / 8 4.7 / 15.9 to 3.8 / 12.9 ms),
// the compiler's own choice below (eight waves there cost Chung-Lu 1M k = 6 0.33 to
// 0.51 ms).
constexpr int wave_waves_per_eu(int k) { return k >= 7 ? 8 : 1; }
template <int K, int MODE>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(wave_waves_per_eu(K))))
k_count_wave(CountParams p) {
    __shared__ WaveSmem<K> sm_all[WAVES];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WaveSmem<K> &sm = sm_all[wave];
    const uint32_t chunk = queue_chunk(p.count, gridDim.x * WAVES, p.chunk_div);
    const bool single = p.per_root != nullptr || (p.colored && p.scheme == KC_COLOR_GLOBAL);
    uint64_t wave_total = 0, acc = 0;
    int ovf = 0;
    uint32_t cb = 0, cn = 0, ci = 0;  // chunk start, size, next unpacked root
    uint32_t my_u = 0, my_d = 0;      // lane t holds root t of the chunk
    uint32_t my_g = 0;
    uint64_t my_base = 0;
    uint32_t cur_g = 0;               // graph whose cliques acc holds (batches)
    const uint32_t home = (blockIdx.x * WAVES + wave) % QCTR;
    uint32_t dead = 0;

    for (;;) {
        if (ci >= cn) {
            const uint32_t b = next_chunk(p.next, p.count, chunk, home, dead);
            if (b == 0xFFFFFFFFu) break;
            cb = b;
            cn = (p.count - b) < chunk ? (p.count - b) : chunk;
            ci = 0;
            my_d = 0;
            if (lane < cn) {
                my_u = p.queue[cb + lane];
                my_base = p.optr[my_u];
                my_d = (uint32_t)(p.optr[my_u + 1] - my_base);
                my_g = p.graph_of ? p.graph_of[my_u] : 0u;
            }
        }
        // pack roots ci, ci+1, ... of one graph while their out-degrees sum to at most 64
        const uint32_t pg = __shfl(my_g, ci, 64);
        if (pg != cur_g) {
            const uint64_t part = kc_wave_sum_checked(acc, &ovf);
            acc = 0;
            if (lane == 0) add_to(p, cur_g, part, ovf, blockIdx.x * WAVES + wave);
            cur_g = pg;
        }
        // the pack is a run of the chunk that stays in graph pg
        const uint64_t other = __ballot(lane >= ci && lane < cn && my_g != pg);
        const uint32_t run_end = other ? (uint32_t)__builtin_ctzll(other) : cn;
        const bool cand = lane >= ci && lane < run_end;
        const uint32_t dl = cand ? my_d : 0u;
        const uint32_t incl = kc_wave_incl_u32(dl);
        const uint32_t before = __shfl(incl - dl, ci, 64);  // sum below root ci
        uint32_t g = (uint32_t)__popcll(__ballot(cand && incl - before <= 64u));
        if (single || g == 0) g = 1;
        const uint32_t S = __shfl(incl, ci + g - 1, 64) - before;  // lanes used
        if (lane >= ci && lane < ci + g) sm.rstart[lane - ci] = incl - dl - before;
        kc_wave_sync();
        uint32_t r = 0;  // packed root of this lane
        if (lane < S) r = kc_seg_find(sm.rstart, g, lane);
        const uint32_t rl = ci + r;
        const uint32_t u = __shfl(my_u, rl, 64);
        const uint64_t rbase = __shfl(my_base, rl, 64);
        const uint32_t rd = __shfl(my_d, rl, 64);
        const uint32_t r0 = lane < S ? sm.rstart[r] : 0u;
        ci += g;
        uint32_t d = S;

        if (MODE == MODE_CACHED) {
            // G+(u) rows from the staged cache, shifted into the root's block;
            // colourings drop the edges they exclude
            const bool mine = lane < S;
            uint64_t row = mine ? p.lrows[rbase + (lane - r0)] << r0 : 0ull;
            if (p.colored) {
                const uint32_t a = mine ? p.ocol[rbase + (lane - r0)] : 0u;
                if (p.scheme == KC_COLOR_GLOBAL) {
                    const uint32_t cu = node_colour(p.seed, p.rank2id[u], p.c);
                    const bool keep = mine && node_colour(p.seed, p.rank2id[a], p.c) == cu;
                    const uint64_t kb = __ballot(keep);
                    row = keep ? (row & kb) : 0ull;
                } else {
                    const uint32_t mc = mine ? root_colour(p.seed, p.rank2id[u], p.rank2id[a], p.c) : 0u;
                    sm.colr[lane] = mc;
                    kc_wave_sync();
                    uint64_t x = row, kept = 0;
                    while (x) {
                        const uint32_t j = (uint32_t)__builtin_ctzll(x);
                        x &= x - 1;
                        if (sm.colr[j] == mc) kept |= 1ull << j;
                    }
                    row = kept;
                }
            }
            sm.A.rows[lane] = row;
        } else {
            // Gamma+ lists into LDS; optionally cut to u's colour (global scheme, one root)
            uint32_t a = lane < S ? p.ocol[rbase + (lane - r0)] : 0xFFFFFFFFu;
            if (p.colored && p.scheme == KC_COLOR_GLOBAL) {
                const uint32_t cu = node_colour(p.seed, p.rank2id[u], p.c);
                const bool keep = lane < d && node_colour(p.seed, p.rank2id[a], p.c) == cu;
                const uint64_t bal = __ballot(keep);
                const uint32_t idx = (uint32_t)__popcll(bal & kc_lanemask_lt());
                sm.nb[lane] = 0xFFFFFFFFu;
                kc_wave_sync();
                if (keep) sm.nb[idx] = a;
                kc_wave_sync();
                d = (uint32_t)__popcll(bal);
                a = sm.nb[lane];
            }
            sm.nb[lane] = a;
            const uint32_t lhi = lane < d ? (single ? d : r0 + rd) : 0u;
            sm.blo[lane] = (uint8_t)(lane < d ? r0 : 0u);
            sm.bhi[lane] = (uint8_t)lhi;
            uint32_t len = 0;
            uint64_t ob = 0;
            if (lane < d) {
                ob = p.optr[a];
                len = (uint32_t)(p.optr[a + 1] - ob);
            }
            // only elements from the next member a_{i+1} of the block up to its largest
            // rank can match: cut each sorted out-list to that range (two binary
            // liftings side by side, when an end is beyond); the block's last node
            // has no later member
            const uint32_t bmax = __shfl(a, (lhi ? lhi - 1u : 0u) & 63u, 64);
            const uint32_t bnext = __shfl(a, (lane + 1u) & 63u, 64);
            if (lane + 1u >= lhi) len = 0;
            if (len) {
                const uint32_t *row = p.ocol + ob;
                if (row[len - 1] > bmax || row[0] < bnext) {
                    uint32_t bh = 0, bl = 0;  // elements <= bmax, elements < bnext
                    for (uint32_t st = 1u << (31 - __builtin_clz(len)); st; st >>= 1) {
                        if (bh + st <= len && row[bh + st - 1] <= bmax) bh += st;
                        if (bl + st <= len && row[bl + st - 1] < bnext) bl += st;
                    }
                    ob += bl;
                    len = bh > bl ? bh - bl : 0u;
                }
            }
            const uint32_t sincl = kc_wave_incl_u32(len);
            const uint32_t excl = sincl - len;
            const uint32_t Ttot = __shfl(sincl, 63, 64);
            sm.delta[lane] = ob - excl;
            sm.A.rows[lane] = 0;
            sm.S.filt[lane] = 0;
#pragma unroll
            for (uint32_t h = 0; h < STAGE_WINDOWS; ++h) sm.S.flag[64 * h + lane] = 0;
            const bool percol = p.colored && p.scheme == KC_COLOR_PER_ROOT;
            if (percol) sm.colr[lane] = lane < d ? root_colour(p.seed, p.rank2id[u], p.rank2id[a], p.c) : 0u;
            kc_wave_sync();
            if (lane < d) {
                const uint32_t h = filt_hash(a);
                atomicOr(&sm.S.filt[h >> 5], 1u << (h & 31u));
            }
            kc_wave_sync();

            // staging: row i bit j = [a_j in Gamma+(a_i)], j inside i's block.  The
            // flattened out-lists are read 64 elements per step; the list of each
            // element is the last one starting at or before it (window start flags
            // and a ballot); the filter drops most non-members, the rest queue up
            // for an exact search 64 at a time.
            uint32_t carry = 0, qh = 0, qt = 0;
            // STAGE_WINDOWS windows per step, so that each lane has that many loads in flight
            const uint64_t le_mask = kc_lanemask_lt() | (1ull << lane);
            for (uint32_t w0 = 0; w0 < Ttot; w0 += 64u * STAGE_WINDOWS) {
                if (len && excl >= w0 && excl - w0 < 64u * STAGE_WINDOWS) sm.S.flag[excl - w0] = (uint8_t)(lane + 1u);
                kc_wave_sync();
                uint32_t iw[STAGE_WINDOWS], yw[STAGE_WINDOWS];
#pragma unroll
                for (uint32_t h = 0; h < STAGE_WINDOWS; ++h) {
                    const uint32_t f = sm.S.flag[64 * h + lane];
                    const uint64_t le = __ballot(f != 0) & le_mask;
                    const uint32_t fo = __shfl(f, le ? 63u - (uint32_t)__builtin_clzll(le) : 0u, 64);
                    iw[h] = le ? fo - 1u : carry;
                    carry = __shfl(iw[h], 63, 64);
                    if (f) sm.S.flag[64 * h + lane] = 0;
                }
#pragma unroll
                for (uint32_t h = 0; h < STAGE_WINDOWS; ++h) {
                    const uint32_t e = w0 + 64u * h + lane;
                    yw[h] = e < Ttot ? p.ocol[sm.delta[iw[h]] + e] : 0u;
                }
#pragma unroll
                for (uint32_t h = 0; h < STAGE_WINDOWS; ++h) {
                    const uint32_t y = yw[h];
                    bool keep = false;
                    if (w0 + 64u * h + lane < Ttot) {
                        const uint32_t hs = filt_hash(y);
                        keep = (sm.S.filt[hs >> 5] >> (hs & 31u)) & 1u;
                    }
                    const uint64_t kb = __ballot(keep);
                    if (keep) {
                        const uint32_t slot = (qt + (uint32_t)__popcll(kb & kc_lanemask_lt())) & 127u;
                        sm.S.qy[slot] = y;
                        sm.S.qi[slot] = (uint8_t)iw[h];
                    }
                    qt += (uint32_t)__popcll(kb);
                    if (qt - qh >= 64u) {
                        kc_wave_sync();
                        wave_stage_check(sm, qh, 64u, percol);
                        qh += 64u;
                        kc_wave_sync();
                    }
                }
            }
            if (qt != qh) {
                kc_wave_sync();
                wave_stage_check(sm, qh, qt - qh, percol);
            }
        }
        if (MODE == MODE_STORE) {
            // keep the staged rows (root-local bit positions) for later counts
            kc_wave_sync();
            if (lane < d) {
                const uint64_t row = sm.A.rows[lane] >> r0;
                p.lrows[rbase + (lane - r0)] = row;
                acc += (uint64_t)__popcll(row);  // the root's triangles (q_3), for free
            }
            kc_wave_sync();
            continue;
        }
        kc_wave_sync();
        local_count<LC_REG_WAVE, true, wave_inplace(K)>(sm.A, d, K - 1, acc);

        if (p.per_root) {
            const uint64_t q = kc_wave_sum_checked(acc, &ovf);
            acc = 0;
            if (lane == 0) {
                p.per_root[p.rank2id[u]] = q;
                const uint64_t nt = wave_total + q;
                if (nt < wave_total) ovf = 1;
                wave_total = nt;
            }
        }
        kc_wave_sync();
    }
    // per-lane sums of many roots: one exact, carry-checked reduction at the end
    const uint64_t rest = kc_wave_sum_checked(acc, &ovf);
    if (lane == 0) {
        const uint64_t nt = wave_total + rest;
        if (nt < wave_total) ovf = 1;
        add_to(p, cur_g, nt, ovf, blockIdx.x * WAVES + wave);
    }
}

// ============================================================================
// Workgroup and scratch tiers: packed upper-triangular bitmap.
// Row i holds words (i+1)/64 .. W-1; its first word sits at
// rowoff(i) = i*W - sum_{t=1}^{i} floor(t/64).
// ============================================================================
__host__ __device__ inline uint64_t tri_rowoff(uint64_t i, uint64_t W) { return kc_tri_rowoff(i, W); }
__host__ __device__ inline uint64_t tri_words(uint64_t d) {
    const uint64_t W = (d + 63) / 64;
    return tri_rowoff(d, W);
}

// static LDS of the workgroup kernel: one local-graph area per wave (two-word
// areas from k = 6 on, where candidate sets of 65..128 nodes are compacted; at k = 5
// such a set's count is its triangles, which wide_triangles takes without a local
// graph, and the one-word areas leave room for more blocks per CU) plus small arrays
// the workgroup tier counts at most (k-2)-cliques in a local graph: k-5 stack entries
template <int K>
struct WgAreas {
    static constexpr int NS = K > 5 ? K - 5 : 1;
    using A1 = LocalArea<NS>;
    using A2 = LocalArea2<NS>;
};
__host__ __device__ constexpr size_t wg_local_bytes_k(int K, size_t a1, size_t a2) { return K >= 6 ? a2 : a1; }
template <int K>
__host__ __device__ constexpr size_t wg_local_bytes() {
    return wg_local_bytes_k(K, sizeof(typename WgAreas<K>::A1), sizeof(typename WgAreas<K>::A2));
}
__host__ __device__ inline size_t wg_local_bytes(int K) {
    switch (K) {
        case 3: return wg_local_bytes<3>();
        case 4: return wg_local_bytes<4>();
        case 5: return wg_local_bytes<5>();
        case 6: return wg_local_bytes<6>();
        case 7: return wg_local_bytes<7>();
        case 8: return wg_local_bytes<8>();
        case 9: return wg_local_bytes<9>();
        default: return wg_local_bytes<10>();
    }
}
// static LDS of the workgroup kernel with nw waves per block
__host__ __device__ inline size_t wg_static_lds(int K, int nw = WAVES) { return wg_local_bytes(K) * nw + 128; }

// Layout of one workgroup's arena (LDS, or a global slice for the scratch tier)
// for out-degree cap D, clique size K and nw waves per block.  A count from the
// staged cache needs only the wide stacks and the bitmap, plus the out-list and
// colour arrays when it applies a colouring (lean = 1: cached, uncoloured; 2: cached,
// coloured; 0: staging).  Fields a layout leaves out point at offset 0 and are not
// read.
struct WgLayout {
    size_t nb, seg, colr, delta, stk, htab, bm, bytes;
    uint32_t W, hbits;
};
__host__ __device__ inline WgLayout wg_layout(uint32_t D, int K, int nw = WAVES, int lean = 0) {
    WgLayout L;
    const uint32_t W = (D + 63) / 64;
    const int levels = K > 3 ? K - 3 : 1;  // wide depth-first stack entries
    L.W = W;
    L.hbits = hash_bits(D);
    size_t o = 0;
    L.nb = L.seg = L.colr = L.delta = 0;
    L.htab = (size_t)-1;
    if (lean != 1) {
        L.nb = o;    o += (size_t)D * 4;
        L.seg = o;   o += ((size_t)D + 1) * 4;
        L.colr = o;  o += (size_t)D * 4;
        o = (o + 3) & ~(size_t)3;
    }
    if (lean == 0) {
        // the table lives in the per-wave local-graph areas (idle while staging) when it fits
        const size_t hbytes = ((size_t)1 << L.hbits) * 2;
        L.htab = hbytes <= wg_local_bytes(K) * nw ? (size_t)-1 : o;
        if (L.htab != (size_t)-1) o += hbytes;
        o = (o + 7) & ~(size_t)7;
        L.delta = o; o += (size_t)D * 8;
    }
    o = (o + 7) & ~(size_t)7;
    L.stk = o;   o += (size_t)nw * levels * W * 8;
    L.bm = o;    o += tri_words(D) * 8;
    L.bytes = o;
    return L;
}

// the layout a launch of the given mode uses
__host__ __device__ inline int wg_lean(int mode, bool colored) {
    return mode == MODE_CACHED ? (colored ? 2 : 1) : 0;
}

__device__ __forceinline__ const uint64_t *bm_row(const uint64_t *bm, uint32_t i, uint32_t W) {
    return bm + tri_rowoff(i, W) - ((i + 1) >> 6);  // indexed by absolute word number
}

// Local index of the node at bit b of word l of a node set P: the members are
// numbered in ascending order, so it is the number of members before it.
// `run` holds the members in words lo..l-1.
__device__ __forceinline__ uint32_t member_rank(uint64_t pw, uint32_t b, uint32_t run) {
    return run + (uint32_t)__popcll(pw & ((1ull << b) - 1ull));
}

// Compact the node set P (words lo..W-1, absolute word index) of at most 64
// nodes into A: member t = t-th node of P, local row t = its row restricted to P
// (bits renumbered by member rank, arithmetic only).  Returns the number of members.
template <class Area>
__device__ __forceinline__ uint32_t compact_local(const uint64_t *P, uint32_t lo, uint32_t W, const uint64_t *bm,
                                                  uint32_t Wbm, Area &A) {
    const uint32_t lane = kc_lane();
    uint32_t nmem = 0;
    for (uint32_t l = lo; l < W; ++l) {
        const uint64_t word = P[l];
        if ((word >> lane) & 1ull) A.members[nmem + (uint32_t)__popcll(word & kc_lanemask_lt())] = 64 * l + lane;
        nmem += (uint32_t)__popcll(word);
    }
    kc_wave_sync();
    uint64_t lrow = 0;
    if (lane < nmem) {
        const uint32_t v = A.members[lane];
        const uint64_t *rv = bm_row(bm, v, Wbm);
        const uint32_t vlo = (v + 1) >> 6;
        uint32_t run = 0;
        for (uint32_t l = lo; l < W; ++l) {
            const uint64_t pw = P[l];
            if (l >= vlo) {
                uint64_t x = rv[l] & pw;
                while (x) {
                    const uint32_t b = (uint32_t)__builtin_ctzll(x);
                    x &= x - 1;
                    lrow |= 1ull << member_rank(pw, b, run);
                }
            }
            run += (uint32_t)__popcll(pw);
        }
    }
    A.rows[lane] = lrow;
    kc_wave_sync();
    return nmem;
}

// As compact_local, for a node set of at most 128 nodes into a two-word local graph.
template <class Area>
__device__ __forceinline__ uint32_t compact_local2(const uint64_t *P, uint32_t lo, uint32_t W, const uint64_t *bm,
                                                   uint32_t Wbm, Area &A) {
    const uint32_t lane = kc_lane();
    uint32_t nmem = 0;
    for (uint32_t l = lo; l < W; ++l) {
        const uint64_t word = P[l];
        if ((word >> lane) & 1ull) A.members[nmem + (uint32_t)__popcll(word & kc_lanemask_lt())] = 64 * l + lane;
        nmem += (uint32_t)__popcll(word);
    }
    kc_wave_sync();
    for (uint32_t half = 0; half < 2; ++half) {
        const uint32_t t = lane + 64 * half;
        uint64_t l0 = 0, l1 = 0;
        if (t < nmem) {
            const uint32_t v = A.members[t];
            const uint64_t *rv = bm_row(bm, v, Wbm);
            const uint32_t vlo = (v + 1) >> 6;
            uint32_t run = 0;
            for (uint32_t l = lo; l < W; ++l) {
                const uint64_t pw = P[l];
                if (l >= vlo) {
                    uint64_t x = rv[l] & pw;
                    while (x) {
                        const uint32_t b = (uint32_t)__builtin_ctzll(x);
                        x &= x - 1;
                        const uint32_t li = member_rank(pw, b, run);
                        if (li < 64) l0 |= 1ull << li;
                        else l1 |= 1ull << (li - 64);
                    }
                }
                run += (uint32_t)__popcll(pw);
            }
        }
        A.rows[t][0] = l0;
        A.rows[t][1] = l1;
    }
    kc_wave_sync();
    return nmem;
}

// Members of the node set C (words lo..W-1, absolute word index) gathered 64 at a
// time into mem (one per lane); body(k) runs on each full batch and on the last
// partial one, with lanes 0..k-1 holding members.  (fpart, fparts): only members v
// with v % fparts == fpart are gathered.
template <class Body>
__device__ __forceinline__ void wide_members(const uint64_t *C, uint32_t lo, uint32_t W, uint32_t *mem,
                                             uint32_t fpart, uint32_t fparts, Body body) {
    const uint32_t lane = kc_lane();
    auto flush = [&](uint32_t k) {
        kc_wave_sync();
        body(k);
        kc_wave_sync();
    };
    uint32_t cnt = 0;
    uint64_t cls = ~0ull;  // members of the filter's class in this word
    for (uint32_t wb = lo; wb < W; ++wb) {
        if (fparts > 1) cls = __ballot((64u * wb + lane) % fparts == fpart);
        const uint64_t word = C[wb] & cls;
        if (!word) continue;
        const uint32_t nbits = (uint32_t)__popcll(word);
        const bool bit = (word >> lane) & 1ull;
        const uint32_t rk = cnt + (uint32_t)__popcll(word & kc_lanemask_lt());
        if (bit && rk < 64) mem[rk] = 64 * wb + lane;
        if (cnt + nbits >= 64) {
            flush(64);
            if (bit && rk >= 64) mem[rk - 64] = 64 * wb + lane;
            cnt = cnt + nbits - 64;
        } else {
            cnt += nbits;
        }
    }
    if (cnt) flush(cnt);
}

// Edges of G+(u) inside the node set C: sum over members v of |C n row_v|, each
// lane intersecting its member's row with C.
__device__ __forceinline__ void wide_edges(const uint64_t *C, uint32_t lo, uint32_t W, const uint64_t *bm,
                                           uint32_t *mem, uint64_t &acc, uint32_t fpart = 0, uint32_t fparts = 1) {
    const uint32_t lane = kc_lane();
    wide_members(C, lo, W, mem, fpart, fparts, [&](uint32_t k) {
        if (lane < k) {
            const uint32_t v = mem[lane];
            const uint64_t *rv = bm_row(bm, v, W);
            for (uint32_t l = (v + 1) >> 6; l < W; ++l) acc += (uint64_t)__popcll(rv[l] & C[l]);
        }
    });
}

// Triangles of G+(u) inside the node set C (the count of a set whose members still
// need three nodes): sum over members v, and over w in C n row_v, of
// |C n row_v n row_w|.  Each lane takes one member v and walks its w itself, so no
// step waits for the whole wave.
__device__ __forceinline__ void wide_triangles(const uint64_t *C, uint32_t lo, uint32_t W, const uint64_t *bm,
                                               uint32_t *mem, uint64_t &acc, uint32_t fpart = 0,
                                               uint32_t fparts = 1) {
    const uint32_t lane = kc_lane();
    wide_members(C, lo, W, mem, fpart, fparts, [&](uint32_t k) {
        if (lane < k) {
            const uint32_t v = mem[lane];
            const uint64_t *rv = bm_row(bm, v, W);
            uint32_t c = 0;
            for (uint32_t l = (v + 1) >> 6; l < W; ++l) {
                uint64_t x = C[l] & rv[l];
                while (x) {
                    const uint32_t w = 64 * l + (uint32_t)__builtin_ctzll(x);
                    x &= x - 1;
                    // word l: the members of C n row_v after w are what is left of x;
                    // row w starts at word (w + 1) / 64, so it is read there only when
                    // x still holds bits (w is then not the word's last bit)
                    const uint64_t *rw = bm_row(bm, w, W);
                    if (x) c += (uint32_t)__popcll(x & rw[l]);
                    for (uint32_t l3 = l + 1; l3 < W; ++l3) c += (uint32_t)__popcll(C[l3] & rv[l3] & rw[l3]);
                }
            }
            acc += c;
        }
    });
}

// NW waves per block (4, 8 or 16): the waves share the root's bitmap, so a larger
// block keeps more waves resident when one arena fills most of the LDS.
// L2: the item list holds two-level items (and roots that leave wide nodes to them);
// without it the kernel carries none of that code or its registers.
// Waves per SIMD the register allocation of the workgroup kernel is held to (the
// compiler's own choice gives 141 VGPRs at k = 8, three waves per SIMD).  Measured on
// planted 4M: four waves at k = 8 (125 VGPRs, no spill) 235 to 228 ms; five at k = 6
// and 7 (a few spilled registers) 39.8 / 132 to 36.7 / 129.5 ms, where five cost time
// at k = 5 (R-MAT 22) and k = 8.
constexpr int wg_waves_per_eu(int k) { return k == 6 || k == 7 ? 5 : 4; }
// Chunks of 64 out-list elements a staging wave loads before using them (memory-level
// parallelism: the pass reads the lists of every member of each G+(u)).  Planted 4M:
// one chunk 22.1 ms for the workgroup tier's staging, four 17.5 ms.
constexpr int STAGE_CHUNKS = 4;
template <int K, bool GLOBAL, int MODE, int NW, bool L2>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(wg_waves_per_eu(K))))
k_count_wg(CountParams p) {
    constexpr uint32_t WGT = NW * 64;
    extern __shared__ __align__(16) unsigned char smem_dyn[];
    __shared__ __align__(16) uint64_t s_lraw[NW][wg_local_bytes<K>() / 8];
    __shared__ uint32_t s_misc[4];
    __shared__ uint64_t s_red[NW];
    __shared__ int s_ovf[NW];
    unsigned char *arena = GLOBAL ? (unsigned char *)(p.gscratch + (size_t)blockIdx.x * p.slice_words) : smem_dyn;
    const WgLayout L = wg_layout(p.dcap, K, NW, wg_lean(MODE, p.colored));
    uint32_t *nb = (uint32_t *)(arena + L.nb);
    uint32_t *seg = (uint32_t *)(arena + L.seg);
    uint32_t *colr = (uint32_t *)(arena + L.colr);
    uint64_t *delta = (uint64_t *)(arena + L.delta);
    uint64_t *bm = (uint64_t *)(arena + L.bm);
    uint16_t *htab = L.htab == (size_t)-1 ? reinterpret_cast<uint16_t *>(&s_lraw[0][0])
                                          : (uint16_t *)(arena + L.htab);
    const uint32_t hbits = L.hbits, hsize = 1u << L.hbits;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t Wc = L.W;
    const int levels = K > 3 ? K - 3 : 1;
    uint64_t *stk = (uint64_t *)(arena + L.stk) + (size_t)wave * levels * Wc;
    using A1T = typename WgAreas<K>::A1;
    using A2T = typename WgAreas<K>::A2;
    A1T &A = *reinterpret_cast<A1T *>(&s_lraw[wave][0]);
    A2T &A2 = *reinterpret_cast<A2T *>(&s_lraw[wave][0]);
    // split items are taken one at a time so that the parts of a root spread over blocks
    const uint32_t chunk = p.items ? 1u : queue_chunk(p.count, gridDim.x, p.chunk_div);
    uint64_t block_total = 0;
    uint32_t cur_g = 0;
    int ovf = 0;
    uint32_t cb = 0, cn = 0, ci = 0;
    const uint32_t home = blockIdx.x % QCTR;  // the queue's counters, as in the one-wave tier
    uint32_t dead = 0;

    for (;;) {
        if (ci >= cn) {
            if (wave == 0) {
                const uint32_t b = next_chunk(p.next, p.count, chunk, home, dead);
                if (lane == 0) s_misc[0] = b;
            }
            __syncthreads();
            cb = s_misc[0];
            __syncthreads();
            if (cb == 0xFFFFFFFFu) break;
            cn = (p.count - cb) < chunk ? (p.count - cb) : chunk;
            ci = 0;
        }
        // items (work_item in kc_internal.h): a root's first-level nodes part, part +
        // parts, ...; or one first-level node v2 whose second-level nodes of class part2
        // (mod parts2) are shared by the block's waves (two levels of splitting)
        uint32_t u, part = 0, parts = 1, v2 = 0, part2 = 0, parts2 = 0, wide_t = 0;
        bool skip_wide = false;
        if (p.items) {
            const uint64_t it = p.items[cb + ci];
            u = (uint32_t)(it >> 32);
            const uint32_t lo = (uint32_t)it;
            if (L2 && (lo & KC_ITEM_LEVEL2)) {
                v2 = lo >> 16;
                part2 = (lo >> 7) & 127u;
                parts2 = lo & 127u;
            } else {
                part = (lo >> 16) & 63u;
                parts = lo & 0xFFu;
                if (L2) {
                    skip_wide = (lo & KC_ITEM_SKIP_WIDE) != 0;
                    wide_t = lo >> 22;
                }
            }
        } else {
            u = p.queue[cb + ci];
        }
        ++ci;
        if (u == 0xFFFFFFFFu) continue;  // padding of an item list
        const uint64_t base = p.optr[u];
        uint32_t d = (uint32_t)(p.optr[u + 1] - base);

        uint32_t W;
        uint64_t words;
        if (MODE == MODE_CACHED) {
            // G+(u) from the staged cache; colourings drop the edges they exclude
            W = (d + 63) / 64;
            words = tri_words(d);
            // a root at or below the one-wave limit (promoted to this tier by the learned
            // schedule) keeps one row per node, which is its packed bitmap for d <= 64
            const uint64_t *src = d <= p.stage_wd ? p.lrows + base : p.wbits + p.woff[u];
            for (uint64_t w = tid; w < words; w += WGT) bm[w] = src[w];
            if (p.colored) {
                for (uint32_t t = tid; t < d; t += WGT) nb[t] = p.ocol[base + t];
                __syncthreads();
                if (p.scheme == KC_COLOR_GLOBAL) {
                    // nodes of u's colour; rows of the others and edges to them vanish
                    const uint32_t cu = node_colour(p.seed, p.rank2id[u], p.c);
                    for (uint32_t t = tid; t < d; t += WGT)
                        colr[t] = node_colour(p.seed, p.rank2id[nb[t]], p.c) == cu ? 1u : 0u;
                    __syncthreads();
                    for (uint32_t l = tid; l < W; l += WGT) {  // keep mask, word l, as two halves in seg
                        uint64_t km = 0;
                        for (uint32_t b = 0; b < 64 && 64 * l + b < d; ++b)
                            if (colr[64 * l + b]) km |= 1ull << b;
                        seg[2 * l] = (uint32_t)km;
                        seg[2 * l + 1] = (uint32_t)(km >> 32);
                    }
                    __syncthreads();
                    for (uint32_t i = tid; i < d; i += WGT) {
                        uint64_t *ri = bm + tri_rowoff(i, W) - ((i + 1) >> 6);
                        const bool ki = colr[i] != 0u;
                        for (uint32_t l = (i + 1) >> 6; l < W; ++l)
                            ri[l] = ki ? ri[l] & ((uint64_t)seg[2 * l] | ((uint64_t)seg[2 * l + 1] << 32)) : 0ull;
                    }
                } else {
                    // edges whose two ends differ in colour vanish
                    for (uint32_t t = tid; t < d; t += WGT)
                        colr[t] = root_colour(p.seed, p.rank2id[u], p.rank2id[nb[t]], p.c);
                    __syncthreads();
                    for (uint32_t i = tid; i < d; i += WGT) {
                        uint64_t *ri = bm + tri_rowoff(i, W) - ((i + 1) >> 6);
                        const uint32_t ci0 = colr[i];
                        for (uint32_t l = (i + 1) >> 6; l < W; ++l) {
                            uint64_t x = ri[l], kept = 0;
                            while (x) {
                                const uint32_t b = (uint32_t)__builtin_ctzll(x);
                                x &= x - 1;
                                if (colr[64 * l + b] == ci0) kept |= 1ull << b;
                            }
                            ri[l] = kept;
                        }
                    }
                }
            }
        } else {
            for (uint32_t t = tid; t < d; t += WGT) nb[t] = p.ocol[base + t];
            __syncthreads();
            if (p.colored && p.scheme == KC_COLOR_GLOBAL) {
                // keep only the nodes of u's colour, preserving order
                const uint32_t cu = node_colour(p.seed, p.rank2id[u], p.c);
                for (uint32_t t = tid; t < d; t += WGT) seg[t] = node_colour(p.seed, p.rank2id[nb[t]], p.c) == cu ? 1u : 0u;
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
            W = (d + 63) / 64;
            // out-degrees of Gamma+(u) and their exclusive prefix
            for (uint32_t t = tid; t < d; t += WGT) {
                const uint32_t x = nb[t];
                seg[t] = (uint32_t)(p.optr[x + 1] - p.optr[x]);
                if (p.colored && p.scheme == KC_COLOR_PER_ROOT) colr[t] = root_colour(p.seed, p.rank2id[u], p.rank2id[x], p.c);
            }
            __syncthreads();
            if (tid < 64) {
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
            words = tri_words(d);
            for (uint64_t w = tid; w < words; w += WGT) bm[w] = 0;
            for (uint32_t h = tid; h < hsize / 2; h += WGT) reinterpret_cast<uint32_t *>(htab)[h] = HEMPTY;
            if (tid == 0) s_misc[3] = 0;
            __syncthreads();
            for (uint32_t t = tid; t < d; t += WGT) hash_insert(htab, hbits, nb[t], t);
            __syncthreads();
            const uint32_t Ttot = seg[d];
            if (d > 0) {
                const uint32_t alast = nb[d - 1];
                if (Ttot >= 32u * d) {
                    // long out-lists: one wave per list, coalesced reads of STAGE_CHUNKS
                    // 64-element chunks at a time (as many loads in flight per wave), stop
                    // past alast
                    for (;;) {
                        uint32_t i = 0;
                        if (lane == 0) i = atomicAdd(&s_misc[3], 1u);
                        i = __shfl(i, 0, 64);
                        if (i >= d) break;
                        const uint64_t b = delta[i] + seg[i];
                        const uint32_t len = seg[i + 1] - seg[i];
                        uint64_t *ri = bm + tri_rowoff(i, W) - ((i + 1) >> 6);
                        for (uint32_t o = 0; o < len; o += 64u * STAGE_CHUNKS) {
                            uint32_t y[STAGE_CHUNKS];
#pragma unroll
                            for (int c = 0; c < STAGE_CHUNKS; ++c) {
                                const uint32_t t = o + 64u * c + lane;
                                y[c] = t < len ? p.ocol[b + t] : 0xFFFFFFFFu;
                            }
#pragma unroll
                            for (int c = 0; c < STAGE_CHUNKS; ++c) {
                                if (y[c] > alast) continue;
                                const uint32_t j = hash_find(htab, hbits, nb, y[c]);
                                if (j == HEMPTY) continue;
                                if (p.colored && p.scheme == KC_COLOR_PER_ROOT && colr[i] != colr[j]) continue;
                                atomicOr((unsigned long long *)(ri + (j >> 6)), 1ull << (j & 63));
                            }
                            // the list is sorted: the rest lies past alast
                            if (!__any(y[STAGE_CHUNKS - 1] <= alast)) break;
                        }
                    }
                } else {
                    for (uint32_t e = tid; e < Ttot; e += WGT) {
                        const uint32_t i = kc_seg_find(seg, d, e);
                        const uint32_t y = p.ocol[delta[i] + e];
                        if (y > alast) continue;
                        const uint32_t j = hash_find(htab, hbits, nb, y);
                        if (j == HEMPTY) continue;
                        if (p.colored && p.scheme == KC_COLOR_PER_ROOT && colr[i] != colr[j]) continue;
                        atomicOr((unsigned long long *)(bm_row(bm, i, W) + (j >> 6)), 1ull << (j & 63));
                    }
                }
            }
        }
        if (MODE == MODE_STORE) {
            // keep the staged bitmap for later counts
            __syncthreads();
            uint64_t *dst = p.wbits + p.woff[u];
            uint32_t ec = 0;
            for (uint64_t w = tid; w < words; w += WGT) {
                dst[w] = bm[w];
                ec += (uint32_t)__popcll(bm[w]);
            }
            // the edges of G+(u) are its triangles (q_3 at u, added to the total) and
            // order later counts' work (heaviest first)
            ec = kc_wave_sum_u32(ec);
            if (lane == 0) s_red[wave] = ec;
            __syncthreads();
            if (tid == 0) {
                uint64_t e = 0;
                for (int w = 0; w < NW; ++w) e += s_red[w];
                if (p.wedges) p.wedges[u] = e > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)e;
                const uint64_t nt = block_total + e;
                if (nt < block_total) ovf = 1;
                block_total = nt;
            }
            __syncthreads();
            continue;
        }
        if (tid == 0) s_misc[2] = 0;
        __syncthreads();

        uint64_t acc = 0;
        if (K == 3 && parts == 1) {
            // q_{u,2} = edges of G+(u) = set bits of the whole bitmap
            for (uint64_t w = tid; w < words; w += WGT) acc += (uint64_t)__popcll(bm[w]);
        } else {
            // first-level nodes; a root split into `parts` items (Section 7: heavy
            // G+(u) shared by several reducers) takes the nodes part, part + parts,
            // part + 2 parts, ... in this item.  One node with a whole wave:
            // fpart, fparts: only second-level nodes of this class (filter of local_count)
            auto one_node = [&](const uint32_t i, const uint32_t fpart, const uint32_t fparts) {
                const uint32_t lo0 = (i + 1) >> 6;
                const uint64_t *ri = bm_row(bm, i, W);
                uint32_t pc = 0;
                for (uint32_t l = lo0 + lane; l < W; l += 64) pc += (uint32_t)__popcll(ri[l]);
                pc = kc_wave_sum_u32(pc);
                if ((int)pc < K - 2) return;
                if (K == 4) {
                    wide_edges(ri, lo0, W, bm, A.members, acc, fpart, fparts);
                    return;
                }
                if (pc <= 64) {
                    const uint32_t sN = compact_local(ri, lo0, W, bm, W, A);
                    local_count<LC_REG_WG, false, false>(A, sN, K - 2, acc, fpart, fparts);
                    return;
                }
                if (K >= 6 && p.local2 && pc <= 128) {
                    const uint32_t sN = compact_local2(ri, lo0, W, bm, W, A2);
                    local_count2(A2, sN, K - 2, acc, fpart, fparts);
                    return;
                }
                if (K == 5) {
                    wide_triangles(ri, lo0, W, bm, A.members, acc, fpart, fparts);
                    return;
                }
                // Wide depth-first search.  stk[depth] holds the candidates not yet
                // visited of a node that still needs K-2-depth nodes; a child that
                // needs 2 more is counted by wide_edges, one of at most 64 nodes as a
                // compacted local graph, a larger one is pushed.
                for (uint32_t l = lo0 + lane; l < W; l += 64) stk[l] = ri[l];
                uint32_t lo[KC_KMAX];
                lo[0] = lo0;
                int depth = 0;
                kc_wave_sync();
                while (depth >= 0) {
                    uint64_t *cur = stk + (size_t)depth * Wc;
                    const int need = (K - 2) - depth;
                    int v = -1;
                    for (uint32_t wb = lo[depth]; wb < W; wb += 64) {
                        const uint32_t l = wb + lane;
                        uint64_t word = l < W ? cur[l] : 0ull;
                        if (depth == 0 && fparts > 1 && word) {
                            // second-level nodes of the filter's class only: bits b of word l
                            // with 64 l + b = fpart (mod fparts)
                            uint64_t cls = 0;
                            for (uint32_t b = (fpart + fparts - (64u * l) % fparts) % fparts; b < 64; b += fparts)
                                cls |= 1ull << b;
                            word &= cls;
                        }
                        const uint64_t bal = __ballot(word != 0);
                        if (bal) {
                            const uint32_t fl = (uint32_t)__builtin_ctzll(bal);
                            const uint64_t wsel = __shfl(word, fl, 64);
                            const uint32_t b = (uint32_t)__builtin_ctzll(wsel);
                            v = (int)((wb + fl) * 64 + b);
                            if (lane == fl) cur[l] &= ~(1ull << b);
                            lo[depth] = wb + fl;
                            break;
                        }
                    }
                    kc_wave_sync();
                    if (v < 0) {
                        --depth;
                        continue;
                    }
                    const int cn = need - 1;  // nodes the child still needs (>= 2)
                    const uint32_t clo = ((uint32_t)v + 1) >> 6;
                    const uint64_t *rv = bm_row(bm, (uint32_t)v, W);
                    uint64_t *nxt = cur + Wc;
                    uint32_t cpc = 0;
                    for (uint32_t l = clo + lane; l < W; l += 64) {
                        const uint64_t x = cur[l] & rv[l];
                        nxt[l] = x;
                        cpc += (uint32_t)__popcll(x);
                    }
                    cpc = kc_wave_sum_u32(cpc);
                    kc_wave_sync();
                    if ((int)cpc < cn) continue;
                    if (cn == 2) {
                        wide_edges(nxt, clo, W, bm, A.members, acc);
                        kc_wave_sync();
                    } else if (cn == 3 && cpc > (K >= 6 && p.local2 ? 128u : 64u)) {
                        wide_triangles(nxt, clo, W, bm, A.members, acc);
                        kc_wave_sync();
                    } else if (cpc <= 64) {
                        const uint32_t sN = compact_local(nxt, clo, W, bm, W, A);
                        local_count<LC_REG_WG, false, false>(A, sN, cn, acc);
                    } else if (K >= 6 && p.local2 && cpc <= 128) {
                        const uint32_t sN = compact_local2(nxt, clo, W, bm, W, A2);
                        local_count2(A2, sN, cn, acc);
                    } else {
                        ++depth;
                        lo[depth] = clo;
                    }
                }
            };
            if (L2 && K >= 4 && parts2) {
                // one first-level node; its second-level nodes of class part2 (mod parts2)
                // are dealt out to the block's waves
                if constexpr (L2) one_node(v2, part2 + wave * parts2, parts2 * NW);
            } else if (K >= 4) {
                // Nodes are taken GRAB at a time.  Those with more than 64 candidates
                // go one by one; the others are packed while their candidate sets
                // sum to at most 64 nodes, side by side as the diagonal blocks of one
                // local graph (no edge joins two blocks), counted in one pass.  At k = 4
                // a node's count is the number of edges inside its candidate set: each
                // member lane counts its own, with no local graph built.
                // Grabs of a split root's item shrink as its nodes run out (guided
                // self-scheduling: an eighth of what is left, 2 to 16 nodes), so the
                // waves of the block finish together; whole roots take 16 at a time.
                constexpr uint32_t GRAB = 16;
                const uint32_t nodes = part < d ? (d - part + parts - 1) / parts : 0u;
                uint8_t *rs = reinterpret_cast<uint8_t *>(&A.members[0]);  // block starts
                uint8_t *rt = rs + 64;                                      // block's slot in the grab
                for (;;) {
                    uint32_t j0 = 0, gsz = 0;
                    if (lane == 0) {
                        const uint32_t seen = __hip_atomic_load(&s_misc[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        const uint32_t left = seen < nodes ? nodes - seen : 0u;
                        gsz = parts == 1 ? GRAB : (left / 8u < 2u ? 2u : (left / 8u > GRAB ? GRAB : left / 8u));
                        j0 = atomicAdd(&s_misc[2], gsz);
                    }
                    j0 = __shfl(j0, 0, 64);
                    gsz = __shfl(gsz, 0, 64);
                    if (part + j0 * parts >= d) break;
                    const uint32_t my_i = part + (j0 + lane) * parts;
                    const bool valid = lane < gsz && my_i < d;
                    uint32_t my_pc = 0;
                    if (valid) {
                        const uint64_t *ri = bm_row(bm, my_i, W);
                        for (uint32_t l = (my_i + 1) >> 6; l < W; ++l) my_pc += (uint32_t)__popcll(ri[l]);
                    }
                    // Nodes whose candidate set held more than wide_t nodes when staged are
                    // left to their two-level items.  The test reads the bitmap as staged,
                    // as the item builder did: a colouring or pair mask may have shrunk the
                    // set in LDS.
                    bool mine = valid;
                    if (L2 && skip_wide && valid) {
                        const uint64_t *rr = p.wbits_raw + p.woff[u] + tri_rowoff(my_i, W) - ((my_i + 1) >> 6);
                        uint32_t raw = 0;
                        for (uint32_t l = (my_i + 1) >> 6; l < W; ++l) raw += (uint32_t)__popcll(rr[l]);
                        mine = raw <= wide_t;
                    }
                    uint64_t big = __ballot(mine && my_pc > 64u);
                    while (big) {
                        const uint32_t t = (uint32_t)__builtin_ctzll(big);
                        big &= big - 1;
                        one_node(__shfl(my_i, t, 64), 0u, 1u);
                    }
                    uint64_t cm = __ballot(mine && my_pc >= (uint32_t)(K - 2) && my_pc <= 64u);
                    while (cm) {
                        const bool in = (cm >> lane) & 1ull;
                        const uint32_t v = in ? my_pc : 0u;
                        const uint32_t incl = kc_wave_incl_u32(v);
                        const uint64_t fit = __ballot(in && incl <= 64u);
                        const uint32_t S = __shfl(incl, 63u - (uint32_t)__builtin_clzll(fit), 64);
                        const uint32_t g = (uint32_t)__popcll(fit);
                        if ((fit >> lane) & 1ull) {
                            const uint32_t r = (uint32_t)__popcll(fit & kc_lanemask_lt());
                            rs[r] = (uint8_t)(incl - v);
                            rt[r] = (uint8_t)lane;
                        }
                        kc_wave_sync();
                        uint64_t lrow = 0;
                        if (lane < S) {
                            uint32_t r = 0, hi = g;  // last block starting at or before this lane
                            while (hi - r > 1) {
                                const uint32_t mid = (r + hi) >> 1;
                                if (rs[mid] <= lane) r = mid; else hi = mid;
                            }
                            const uint32_t base = rs[r];
                            const uint32_t i = part + (j0 + rt[r]) * parts;
                            const uint32_t lo0 = (i + 1) >> 6;
                            const uint64_t *ri = bm_row(bm, i, W);
                            // member: the (lane - base)-th node of row i
                            uint32_t rem = lane - base, l = lo0;
                            uint64_t w = ri[l];
                            for (;;) {
                                const uint32_t c = (uint32_t)__popcll(w);
                                if (rem < c) break;
                                rem -= c;
                                w = ri[++l];
                            }
                            const uint32_t vn = 64 * l + kc_select_bit(w, rem);
                            // its row inside row i, renumbered by rank in row i
                            const uint64_t *rv = bm_row(bm, vn, W);
                            const uint32_t vlo = (vn + 1) >> 6;
                            uint32_t run = base;
                            if (K == 4) {
                                for (uint32_t l2 = vlo; l2 < W; ++l2) acc += (uint64_t)__popcll(rv[l2] & ri[l2]);
                                run = W;  // rows are not built
                            }
                            for (uint32_t l2 = K == 4 ? W : lo0; l2 < W; ++l2) {
                                const uint64_t pw = ri[l2];
                                if (l2 >= vlo) {
                                    uint64_t x = rv[l2] & pw;
                                    while (x) {
                                        const uint32_t bpos = (uint32_t)__builtin_ctzll(x);
                                        x &= x - 1;
                                        lrow |= 1ull << (run + (uint32_t)__popcll(pw & ((1ull << bpos) - 1ull)));
                                    }
                                }
                                run += (uint32_t)__popcll(pw);
                            }
                        }
                        if (K > 4) {
                            A.rows[lane] = lrow;
                            kc_wave_sync();
                            local_count<LC_REG_WG, false, false>(A, S, K - 2, acc);
                        } else {
                            kc_wave_sync();  // rs/rt are rewritten by the next pack
                        }
                        cm &= ~fit;
                    }
                }
            } else {
                for (;;) {
                    uint32_t j = 0;
                    if (lane == 0) j = atomicAdd(&s_misc[2], 1u);
                    j = __shfl(j, 0, 64);
                    const uint32_t i = part + j * parts;
                    if (i >= d) break;
                    one_node(i, 0u, 1u);
                }
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
            for (int w = 0; w < NW; ++w) {
                const uint64_t nq = q + s_red[w];
                if (nq < q || s_ovf[w]) ovf = 1;
                q = nq;
            }
            if (p.per_root) {
                if (parts == 1 && (!L2 || (!skip_wide && !parts2))) p.per_root[p.rank2id[u]] = q;
                else atomicAdd((unsigned long long *)&p.per_root[p.rank2id[u]], (unsigned long long)q);
            }
            const uint32_t gq = p.graph_of ? p.graph_of[u] : 0u;
            if (gq != cur_g) {
                add_to(p, cur_g, block_total, ovf, blockIdx.x);
                block_total = 0;
                cur_g = gq;
            }
            const uint64_t nt = block_total + q;
            if (nt < block_total) ovf = 1;
            block_total = nt;
        }
        __syncthreads();
    }
    if (tid == 0) add_to(p, cur_g, block_total, ovf, blockIdx.x);
}

// ----------------------------------------------------------------------------
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

template <int K, int MODE>
void launch_tiers(const CountParams &base, const kc_queue &q, uint32_t *cursors, const DevInfo &di, hipStream_t s,
                  uint64_t *gscratch, size_t slice_words, uint32_t scratch_blocks, hipEvent_t *ev,
                  hipStream_t side = nullptr, hipEvent_t fork = nullptr, hipEvent_t join = nullptr) {
    const kc_tuning_t &tu = kc_tuning_now();
    // Scratch tier, workgroup tier, then the one-wave tier, on s.  (The one-wave tier
    // beside the others on a second stream was faster at k >= 7 before the workgroup
    // arena shrank for cached counts; now the workgroup tier runs faster alone and
    // the one-wave tier after it in small chunks: planted 4M k = 7 / 8, 138 / 268 ms in
    // sequence against 154 / 286 ms side by side.)  side, fork, join: the third
    // stream for the workgroup tier's large roots (may be null).
    // ev: [0] scratch start, [1] scratch end / workgroup start, [2] workgroup end,
    // [3] all done, [4] [5] the one-wave tier.
    hipStream_t ws = s;
    auto launch_wave = [&]() {
        if (ev) (void)hipEventRecord(ev[4], ws);
        if (q.count[0]) {
            CountParams p = base;
            p.queue = q.ptr[0];
            p.count = q.count[0];
            p.next = cursors + 0;
            uint32_t blocks = (q.count[0] + WAVES - 1) / WAVES;
            uint32_t per_cu = (uint32_t)(tu.wave_blocks_per_cu > 0 ? tu.wave_blocks_per_cu : 8);
            int occ = 0;  // resident blocks per CU (registers, LDS)
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)&k_count_wave<K, MODE>, WG, 0) ==
                    hipSuccess &&
                occ > 0 && (uint32_t)occ < per_cu)
                per_cu = (uint32_t)occ;
            const uint32_t cap = (uint32_t)di.cus * per_cu;
            if (blocks > cap) blocks = cap;
            // Chunk size (queue / (waves x divisor)) by clique size, measured on planted
            // 4M and Chung-Lu 1M: staging takes half-size chunks; counts from the cache
            // smaller chunks as the work per root grows (planted k = 6, 4.2 ms at the
            // base divisor, 1.3 ms at 4x; k = 8, 96 ms at the base, 17 ms at 8x).
            const uint32_t cd = base.chunk_div;
            if (MODE == MODE_STORE) p.chunk_div = cd * 2;
            else if (MODE == MODE_CACHED && K == 5) p.chunk_div = cd * 2;
            else if (MODE == MODE_CACHED && K == 6) p.chunk_div = cd * 4;
            else if (MODE == MODE_CACHED && K >= 7) p.chunk_div = cd * 8;
            hipLaunchKernelGGL((k_count_wave<K, MODE>), dim3(blocks), dim3(WG), 0, ws, p);
        }
        if (ev) (void)hipEventRecord(ev[5], ws);
    };
    if (ev) (void)hipEventRecord(ev[0], s);
    // scratch tier first: the largest roots
    if (q.count[2]) {
        CountParams p = base;
        p.queue = q.ptr[2];
        p.count = q.count[2];
        p.next = cursors + 2;
        p.gscratch = gscratch;
        p.slice_words = slice_words;
        p.dcap = q.max_d[2];
        hipLaunchKernelGGL((k_count_wg<K, true, MODE, WAVES, false>), dim3(scratch_blocks), dim3(WG), 0, s, p);
    }
    if (ev) (void)hipEventRecord(ev[1], s);
    if (q.count[1]) {
        // Block shape of a launch whose arena holds out-degree dmax: waves per block
        // (4, 8 or 16; the wg_waves tunable fixes it) and resident blocks per CU.  Four
        // waves per block while at least four such blocks fit on a CU (the waves of a
        // block share one root or item: small blocks balance better); otherwise the
        // shape with the most waves resident (LDS and registers), at most 32.  One
        // large arena per block (a root of out-degree 1031 takes about 90 KB) leaves
        // room for one block: more waves in it keep the CU busy while others wait on
        // LDS.  Measured: R-MAT 22 at k = 5, 1.98 s with four waves, 1.44 s with the
        // larger block; planted 4M at k = 8, the large roots' launch (three four-wave
        // blocks or two eight-wave blocks per CU): the tier 229 ms with four waves, 204
        // ms with eight; with two four-wave blocks as the bound, k = 5..7 and R-MAT
        // unchanged.
        const void *fn[3] = {(const void *)&k_count_wg<K, false, MODE, 4, false>,
                             (const void *)&k_count_wg<K, false, MODE, 8, false>,
                             (const void *)&k_count_wg<K, false, MODE, 16, false>};
        const void *fn2[3] = {(const void *)&k_count_wg<K, false, MODE, 4, true>,
                              (const void *)&k_count_wg<K, false, MODE, 8, true>,
                              (const void *)&k_count_wg<K, false, MODE, 16, true>};
        const int nws[3] = {4, 8, 16};
        // static LDS of each block shape as compiled (the per-wave arrays grow with it),
        // looked up once; the attribute caps the dynamic LDS of later launches (graph
        // replays included)
        static size_t stat[3] = {0, 0, 0};
        for (int i = 0; i < 3; ++i) {
            if (!stat[i]) {  // the same static arrays with and without L2
                hipFuncAttributes fa;
                stat[i] = hipFuncGetAttributes(&fa, fn[i]) == hipSuccess ? fa.sharedSizeBytes
                                                                          : wg_static_lds(K, nws[i]) + 1024;
            }
            if (stat[i] < di.lds_max) {
                (void)hipFuncSetAttribute(fn[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)(di.lds_max - stat[i]));
                (void)hipFuncSetAttribute(fn2[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)(di.lds_max - stat[i]));
            }
        }
        struct Shape {
            int idx;
            uint32_t per_cu;
        };
        auto shape = [&](uint32_t dmax) {
            Shape best{0, 0};
            for (int i = 0; i < 3; ++i) {
                const int nw = nws[i];
                if (tu.wg_waves && tu.wg_waves != nw) continue;
                const WgLayout L = wg_layout(dmax < 65 ? 65 : dmax, K, nw, wg_lean(MODE, base.colored));
                const size_t per_block = L.bytes + stat[i] + 256;
                if (per_block > di.lds_max) continue;
                uint32_t per_cu = (uint32_t)(di.lds_max / per_block);
                // no more than are resident at once (registers): a block launched past
                // that starts only when the queue is spent
                int occ = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, q.wg_l2 ? fn2[i] : fn[i], nw * 64, L.bytes) ==
                        hipSuccess &&
                    occ > 0 &&
                    (uint32_t)occ < per_cu)
                    per_cu = (uint32_t)occ;
                if (per_cu * (uint32_t)nw > 32u) per_cu = 32u / (uint32_t)nw;
                if (tu.wg_blocks_per_cu > 0 && (uint32_t)tu.wg_blocks_per_cu < per_cu)
                    per_cu = (uint32_t)tu.wg_blocks_per_cu;
                if (i == 0 && per_cu >= 4 && !tu.wg_waves) return Shape{0, per_cu};
                if (per_cu * (uint32_t)nw > best.per_cu * (uint32_t)nws[best.idx]) best = Shape{i, per_cu};
            }
            if (best.per_cu == 0) best = Shape{0, 1};  // every root of the tier fits four waves' arena
            return best;
        };
        auto launch_wg = [&](const uint32_t *queue, uint32_t count, const uint64_t *items, uint32_t *next,
                             uint32_t dmax, bool items_l2, hipStream_t st) {
            CountParams p = base;
            p.queue = queue;
            p.count = count;
            p.items = items;
            p.next = next;
            p.dcap = dmax < 65 ? 65 : dmax;
            const Shape sh = shape(dmax);
            const int nw = nws[sh.idx];
            const WgLayout L = wg_layout(p.dcap, K, nw, wg_lean(MODE, p.colored));
            uint32_t blocks = (uint32_t)di.cus * sh.per_cu;
            if (blocks > count) blocks = count;
            const bool l2 = items && items_l2;
            if (nw == 16 && l2)
                hipLaunchKernelGGL((k_count_wg<K, false, MODE, 16, true>), dim3(blocks), dim3(1024), L.bytes, st, p);
            else if (nw == 16)
                hipLaunchKernelGGL((k_count_wg<K, false, MODE, 16, false>), dim3(blocks), dim3(1024), L.bytes, st, p);
            else if (nw == 8 && l2)
                hipLaunchKernelGGL((k_count_wg<K, false, MODE, 8, true>), dim3(blocks), dim3(512), L.bytes, st, p);
            else if (nw == 8)
                hipLaunchKernelGGL((k_count_wg<K, false, MODE, 8, false>), dim3(blocks), dim3(512), L.bytes, st, p);
            else if (l2)
                hipLaunchKernelGGL((k_count_wg<K, false, MODE, 4, true>), dim3(blocks), dim3(256), L.bytes, st, p);
            else
                hipLaunchKernelGGL((k_count_wg<K, false, MODE, 4, false>), dim3(blocks), dim3(256), L.bytes, st, p);
        };
        if (q.wg_items && q.wg_items2) {
            // the large roots' items with their large arena on the third stream, beside
            // the small roots' items with a small arena (more blocks per CU) on s
            const bool fork_ok = side && fork && join;
            hipStream_t sb = fork_ok ? side : s;
            if (fork_ok) {
                (void)hipEventRecord(fork, s);
                (void)hipStreamWaitEvent(side, fork, 0);
            }
            launch_wg(q.ptr[1], q.wg_item_count, q.wg_items, cursors + 1, q.max_d[1], q.wg_l2, sb);
            if (fork_ok) (void)hipEventRecord(join, side);
            launch_wg(q.ptr[1], q.wg_item_count2, q.wg_items2, cursors + 3 + KC_WG_CLASSES, q.wg_dmax2, q.wg_l2b,
                      s);
            if (fork_ok) (void)hipStreamWaitEvent(s, join, 0);
        } else if (q.wg_items) {
            launch_wg(q.ptr[1], q.wg_item_count, q.wg_items, cursors + 1, q.max_d[1], q.wg_l2, s);
        } else if (q.wg_ncls > 1) {
            // Consecutive out-degree classes (largest first) grouped into launches: a
            // class joins the current group when a launch of its own would hold no
            // more blocks per CU, or when the group is too short to keep the device
            // busy past its tail (fewer than 4 roots per resident block).
            Shape cap = shape(q.wg_cls_dmax[0]);
            uint32_t g0 = 0, cnt = q.wg_cls_cnt[0];
            for (uint32_t c = 1; c <= q.wg_ncls; ++c) {
                if (c < q.wg_ncls) {
                    const Shape sc = shape(q.wg_cls_dmax[c]);
                    if ((sc.idx == cap.idx && sc.per_cu == cap.per_cu) || cnt < 4u * (uint32_t)di.cus * cap.per_cu) {
                        cnt += q.wg_cls_cnt[c];
                        continue;
                    }
                }
                launch_wg(q.ptr[1] + q.wg_cls_off[g0], cnt, nullptr, cursors + 3 + g0, q.wg_cls_dmax[g0], false, s);
                if (c < q.wg_ncls) {
                    g0 = c;
                    cnt = q.wg_cls_cnt[c];
                    cap = shape(q.wg_cls_dmax[c]);
                }
            }
        } else {
            launch_wg(q.ptr[1], q.count[1], nullptr, cursors + 1, q.max_d[1], false, s);
        }
    }
    if (ev) (void)hipEventRecord(ev[2], s);
    launch_wave();
    if (ev) (void)hipEventRecord(ev[3], s);
}

__global__ void k_fill_u64(uint64_t *p, size_t n, uint64_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// *total += the 32 partial totals, carry-checked (one wave)
__global__ void k_total_slots(uint64_t *res) {
    const uint32_t lane = threadIdx.x;
    uint64_t v = lane < 32 ? res[KC_RES_SLOTS + lane] : 0ull;
    int ovf = 0;
    v = kc_wave_sum_checked(v, &ovf);
    if (lane == 0) {
        const uint64_t t = res[0] + v;
        if (t < v || ovf) res[1] = 1ull;
        res[0] = t;
    }
}

// cache words of each root: its packed bitmap when it is above the wave tier
__global__ void k_stage_sizes(const uint64_t *optr, uint32_t n, uint32_t wd, uint64_t *words) {
    const size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint64_t d = optr[x + 1] - optr[x];
    words[x] = d > wd ? tri_words(d) : 0ull;
}

}  // namespace

// Plain pair sampling (Section 6): the pair (x, y) of Gamma+(u), x before y in the
// order, is kept iff (H2 >> 32) < t, H2 = mix64(mix64(seed ^ mix64(u << 32 | x)) ^
// mix64(y)) on original ids; a masked copy of the staged cache is then counted.
__device__ __forceinline__ bool pair_kept(uint64_t seed, uint32_t uid, uint32_t xid, uint32_t yid, uint64_t t) {
    const uint64_t h = kc_mix64(kc_mix64(seed ^ kc_mix64(((uint64_t)uid << 32) | xid)) ^ kc_mix64((uint64_t)yid));
    return (h >> 32) < t;
}

// one-wave tier rows (root-local bits), one thread per row; rows of larger roots are unused
__global__ void k_pair_mask_rows(const uint64_t *optr, const uint32_t *ocol, const uint32_t *rank2id, uint32_t n,
                                 uint64_t m, uint32_t wd, const uint64_t *in, uint64_t *out, uint64_t seed, uint64_t t) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uint32_t lo = 0, hi = n;  // the root owning slot e: the last rank with optr[u] <= e
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (optr[mid] <= e) lo = mid; else hi = mid;
    }
    const uint64_t b = optr[lo], d = optr[lo + 1] - b, i = e - b;
    // only rows of staged roots (2 <= d <= wd) hold data; a root of out-degree 1 is
    // never staged and its slot is uninitialised.  Bits are kept to the row's later
    // members i < j < d, so no read leaves the root's out-list.
    uint64_t x = 0, kept = 0;
    if (d >= 2 && d <= wd) x = in[e] & (d >= 64 ? ~0ull : ((1ull << d) - 1ull)) & ~((2ull << i) - 1ull);  // i < d <= 64
    if (x) {
        const uint32_t uid = rank2id[lo], xid = rank2id[ocol[e]];
        while (x) {
            const uint32_t j = (uint32_t)__builtin_ctzll(x);
            x &= x - 1;
            if (pair_kept(seed, uid, xid, rank2id[ocol[b + j]], t)) kept |= 1ull << j;
        }
    }
    out[e] = kept;
}

// packed bitmaps of the roots above the one-wave tier (the wide part of the degree
// queue), one block per root, one thread per row
__global__ void k_pair_mask_bitmaps(const uint32_t *wide, const uint64_t *optr, const uint32_t *ocol,
                                    const uint32_t *rank2id, const uint64_t *woff, const uint64_t *in, uint64_t *out,
                                    uint64_t seed, uint64_t t) {
    const uint32_t u = wide[blockIdx.x];
    const uint64_t b = optr[u];
    const uint32_t d = (uint32_t)(optr[u + 1] - b), W = (d + 63) / 64;
    const uint32_t uid = rank2id[u];
    for (uint32_t i = threadIdx.x; i < d; i += blockDim.x) {
        const uint32_t xid = rank2id[ocol[b + i]];
        const uint64_t off = woff[u] + tri_rowoff(i, W) - ((i + 1) >> 6);  // word l of row i at off + l
        for (uint32_t l = (i + 1) >> 6; l < W; ++l) {
            // bits of later members only: i < 64 l + bit < d
            const uint32_t hi = d - 64 * l;  // >= 1 since l < W
            uint64_t x = in[off + l] & (hi >= 64 ? ~0ull : ((1ull << hi) - 1ull)), kept = 0;
            if (64 * l <= i) x &= ~((2ull << (i - 64 * l)) - 1ull);
            while (x) {
                const uint32_t bit = (uint32_t)__builtin_ctzll(x);
                x &= x - 1;
                if (pair_kept(seed, uid, xid, rank2id[ocol[b + 64 * l + bit]], t)) kept |= 1ull << bit;
            }
            out[off + l] = kept;
        }
    }
}

kc_status kc_stage_queue(const kc_graph *g, const kc_queue &q, int wd, uint64_t *res, kc_tmp &lrows, kc_tmp &wbits,
                         kc_tmp &woff, bool &cached) {
    cached = false;
    hipStream_t s = g->stream;
    const uint32_t n = g->n;
    // the staging pass runs the clique-size-3 kernels: their workgroup arena must hold
    // every root the queue puts in the workgroup tier
    if (q.count[1] && q.max_d[1] > kc_lds_dcap(g->device, 3)) return KC_OK;
    KC_TRY(kc_tmp_alloc(woff, ((size_t)n + 1) * 8, s));
    {
        kc_tmp sizes;
        KC_TRY(kc_tmp_alloc(sizes, (size_t)(n ? n : 1) * 8, s));
        hipLaunchKernelGGL(k_stage_sizes, dim3((n + 255) / 256), dim3(256), 0, s, (const uint64_t *)g->optr, n,
                           (uint32_t)wd, sizes.as<uint64_t>());
        KC_HIP(hipGetLastError());
        KC_TRY(kc_scan_excl_u64(sizes.as<uint64_t>(), woff.as<uint64_t>(), n, woff.as<uint64_t>() + n, s));
    }
    uint64_t *h = kc_pinned_scratch();
    KC_HIP(hipMemcpyAsync(h, woff.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost, s));
    KC_TRY(kc_sync(s));
    const uint64_t total = h[0];
    size_t fr = 0, tot = 0;
    KC_HIP(hipMemGetInfo(&fr, &tot));
    if ((g->m + total) * 8 > fr / 2) return KC_OK;
    KC_TRY(kc_tmp_alloc(lrows, (size_t)(g->m ? g->m : 1) * 8, s));
    KC_TRY(kc_tmp_alloc(wbits, (size_t)(total ? total : 1) * 8, s));
    kc_graph gs = *g;  // a view with the caches attached (owns nothing)
    gs.lrows = lrows.as<uint64_t>();
    gs.wbits = wbits.as<uint64_t>();
    gs.woff = woff.as<uint64_t>();
    gs.stage_wd = wd;
    kc_tmp gscr;
    size_t slice_words = 0;
    uint32_t scratch_blocks = 0;
    KC_TRY(kc_count_scratch(g, q, 3, gscr, slice_words, scratch_blocks));
    kc_count_args a;
    a.k = 3;
    a.store = 1;
    const kc_status st = kc_count_launch(&gs, q, a, res, nullptr, 0, nullptr, gscr.as<uint64_t>(), slice_words,
                                         scratch_blocks, s, nullptr);
    gs.lrows = gs.wbits = gs.woff = nullptr;
    gs.optr = nullptr;  // the copy must not look like an owner of anything
    KC_TRY(st);
    KC_TRY(kc_sync(s));
    cached = true;
    return KC_OK;
}

// Stage every root's G+(u) into the handle's cache (wave tier split at wd).
// Leaves the handle uncached (staged = -1) when the cache would take more than
// half of the free device memory.
kc_status kc_stage(kc_graph *g, int wd) {
    if (g->staged != 0 && g->stage_wd == wd) return KC_OK;
    hipStream_t s = g->stream;
    kc_cache_free(g->lrows, s);
    kc_cache_free(g->wbits, s);
    kc_cache_free(g->woff, s);
    kc_cache_free(g->wq, s);
    kc_cache_free(g->wq2, s);
    kc_cache_free(g->wedges, s);
    g->lrows = g->wbits = g->woff = nullptr;
    g->wq = g->wq2 = nullptr;
    g->wedges = nullptr;
    g->wq_ready = 0;
    g->staged = 0;
    const uint32_t n = g->n;
    uint64_t *woff = nullptr;
    KC_TRY(kc_dev_alloc((void **)&woff, ((size_t)n + 1) * 8, s));
    {
        kc_tmp sizes;
        KC_TRY(kc_tmp_alloc(sizes, (size_t)(n ? n : 1) * 8, s));
        hipLaunchKernelGGL(k_stage_sizes, dim3((n + 255) / 256), dim3(256), 0, s, (const uint64_t *)g->optr, n,
                           (uint32_t)wd, sizes.as<uint64_t>());
        KC_HIP(hipGetLastError());
        KC_TRY(kc_scan_excl_u64(sizes.as<uint64_t>(), woff, n, woff + n, s));
    }
    // the staging pass runs over the degree queue; its out-degree histogram (on
    // the host) also gives the cache size without reading the scan back
    kc_queue q;
    KC_TRY(kc_build_queue(g, 3, KC_SCHED_DEGREE, kc_lds_dcap(g->device, 3), q));
    uint64_t total = 0;
    if (g->dq_ready && g->dq_wd == wd && g->dq_hist) {
        for (uint32_t d = (uint32_t)wd + 1; d <= g->max_outdeg; ++d) total += g->dq_hist[d] * tri_words(d);
    } else {
        uint64_t *h = kc_pinned_scratch();
        KC_HIP(hipMemcpyAsync(h, woff + n, 8, hipMemcpyDeviceToHost, s));
        KC_TRY(kc_sync(s));
        total = h[0];
    }
    size_t fr = 0, tot = 0;
    KC_HIP(hipMemGetInfo(&fr, &tot));
    if ((g->m + total) * 8 > fr / 2) {
        kc_cache_free(woff, s);
        g->staged = -1;
        g->stage_wd = wd;
        return KC_OK;
    }
    g->woff = woff;
    g->stage_words = total;
    KC_TRY(kc_dev_alloc((void **)&g->wedges, (size_t)(n ? n : 1) * 4, s));
    KC_TRY(kc_dev_alloc((void **)&g->lrows, (size_t)(g->m ? g->m : 1) * 8, s));
    KC_TRY(kc_dev_alloc((void **)&g->wbits, (size_t)(total ? total : 1) * 8, s));
    kc_tmp gscr;
    size_t slice_words = 0;
    uint32_t scratch_blocks = 0;
    KC_TRY(kc_count_scratch(g, q, 3, gscr, slice_words, scratch_blocks));
    kc_count_args a;
    a.k = 3;
    a.store = 1;
    hipEvent_t sev[6] = {g->sev[0], g->sev[1], g->sev[2], g->sev[3], g->sev[4], g->sev[5]};
    KC_TRY(kc_count_launch(g, q, a, g->d_res, nullptr, 0, nullptr, gscr.as<uint64_t>(), slice_words, scratch_blocks,
                           s, sev[0] ? sev : nullptr));
    g->staged = 1;
    g->stage_wd = wd;
    return KC_OK;
}

// Largest out-degree of the workgroup tier: the largest whose workgroup layout
// (packed bitmap included) fits in LDS, or the wg_dmax tunable when that is lower.
uint32_t kc_lds_dcap(int device, int k) {
    const DevInfo di = dev_info(device);
    const size_t budget = di.lds_max - wg_static_lds(k) - 512;
    uint32_t lo = 64, hi = 1 << 16;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        if (wg_layout(mid, k).bytes <= budget) lo = mid; else hi = mid - 1;
    }
    const int cap = kc_tuning_now().wg_dmax;
    if (cap > 0 && (uint32_t)cap < lo) lo = (uint32_t)cap;
    return lo;
}

size_t kc_scratch_slice_words(uint32_t dmax, int k) { return (wg_layout(dmax, k).bytes + 7) / 8; }

// Four-wave workgroup blocks per CU that LDS allows when the arena holds out-degree d
// (an uncoloured count from the staged cache).
uint32_t kc_wg_blocks_per_cu(int device, int k, uint32_t d) {
    const DevInfo di = dev_info(device);
    const size_t per_block = wg_layout(d < 65 ? 65 : d, k, 4, wg_lean(MODE_CACHED, false)).bytes +
                             wg_static_lds(k, 4) + 1024;
    return (uint32_t)(di.lds_max / per_block);
}

// Global-memory slices of the scratch tier for this queue.
kc_status kc_count_scratch(const kc_graph *g, const kc_queue &q, int k, kc_tmp &gscr, size_t &slice_words,
                           uint32_t &blocks) {
    const DevInfo di = dev_info(g->device);
    slice_words = 0;
    blocks = 0;
    if (!q.count[2]) return KC_OK;
    slice_words = kc_scratch_slice_words(q.max_d[2], k);
    blocks = q.count[2] < (uint32_t)di.cus ? q.count[2] : (uint32_t)di.cus;
    while (blocks > 1 && slice_words * 8 * blocks > (8ull << 30)) blocks /= 2;  // at most 8 GiB
    return kc_tmp_alloc(gscr, slice_words * 8 * blocks, g->stream);
}

// The counting kernels of one queue, enqueued on s with no allocation, no
// synchronisation and no memset (so the sequence can be captured in a graph).
// res (KC_RES_WORDS words): [0] total, [1] overflow flag, then u32 queue counters, each
// queue's QCTR of them QCTR_STRIDE apart from its first (spent flags QCTR_FLAG further):
// wave tier at 0, workgroup at 1, scratch at 2, workgroup classes at 3 + c; gtotals/graph_of
// for batches.
kc_status kc_count_launch(const kc_graph *g, const kc_queue &q, const kc_count_args &a, uint64_t *res,
                          unsigned long long *gtotals, uint32_t ngraphs, const uint32_t *graph_of, uint64_t *gscratch,
                          size_t slice_words, uint32_t scratch_blocks, hipStream_t s, hipEvent_t *tier_ev,
                          bool use_side) {
    hipStream_t side = use_side ? g->side : nullptr;
    const DevInfo di = dev_info(g->device);
    hipLaunchKernelGGL(k_fill_u64, dim3((KC_RES_WORDS + 63) / 64), dim3(64), 0, s, res, (size_t)KC_RES_WORDS, 0ull);
    if (gtotals)
        hipLaunchKernelGGL(k_fill_u64, dim3((ngraphs + 255) / 256), dim3(256), 0, s, (uint64_t *)gtotals,
                           (size_t)ngraphs, 0ull);
    // test hook, read once per process: the total starts at this value, which forces the
    // carry check of the reduction
    static const char *const bias = getenv("KC_TEST_TOTAL_BIAS");
    if (bias && !gtotals)
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, res, (size_t)1, (uint64_t)strtoull(bias, nullptr, 0));
    CountParams p{};
    p.optr = g->optr;
    p.ocol = g->ocol;
    p.rank2id = g->rank2id;
    p.per_root = a.per_root;
    p.total = (unsigned long long *)res;
    p.slots = (unsigned long long *)(res + KC_RES_SLOTS);
    p.overflow = (uint32_t *)(res + 1);
    p.colored = a.colored;
    p.scheme = a.scheme;
    p.c = a.c;
    p.seed = a.seed;
    p.chunk_div = (uint32_t)(kc_tuning_now().chunk_div > 0 ? kc_tuning_now().chunk_div : 8);
    p.local2 = kc_tuning_now().local_bits >= 128 ? 1u : 0u;
    p.graph_of = graph_of;
    p.gtotals = gtotals;
    p.lrows = g->lrows;
    p.wbits = g->wbits;
    p.stage_wd = (uint32_t)g->stage_wd;
    p.wbits_raw = g->wbits_raw ? g->wbits_raw : g->wbits;
    p.woff = g->woff;
    p.wedges = g->wedges;
    uint32_t *cursors = (uint32_t *)(res + 2);
    if (a.store) {
        // staging into the cache does not depend on k; its total is q_3 (the edges of
        // every G+(u)), kept in res as a count would leave it
        launch_tiers<3, MODE_STORE>(p, q, cursors, di, s, gscratch, slice_words, scratch_blocks, tier_ev);
        if (!gtotals) hipLaunchKernelGGL(k_total_slots, dim3(1), dim3(64), 0, s, res);
        KC_HIP(hipGetLastError());
        return KC_OK;
    }
    switch (a.k) {
#define KC_CASE(KK)                                                                                          \
    case KK:                                                                                                 \
        if (a.cached)                                                                                        \
            launch_tiers<KK, MODE_CACHED>(p, q, cursors, di, s, gscratch, slice_words, scratch_blocks, tier_ev, \
                                          side, g->fork, g->join);                                           \
        else                                                                                                 \
            launch_tiers<KK, MODE_STAGE>(p, q, cursors, di, s, gscratch, slice_words, scratch_blocks, tier_ev); \
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
    if (!gtotals) hipLaunchKernelGGL(k_total_slots, dim3(1), dim3(64), 0, s, res);
    KC_HIP(hipGetLastError());
    return KC_OK;
}

// Tier kernel times of the staging pass that just ran (after a host synchronisation).
static void stage_tier_times(kc_graph *g) {
    float tt[3] = {0.f, 0.f, 0.f};
    if (g->sev[0]) {
        (void)hipEventElapsedTime(&tt[2], g->sev[0], g->sev[1]);
        (void)hipEventElapsedTime(&tt[1], g->sev[1], g->sev[2]);
        (void)hipEventElapsedTime(&tt[0], g->sev[4], g->sev[5]);
    }
    for (int t = 0; t < 3; ++t) g->t_stage_tier[t] = tt[t];
}

kc_status kc_count_impl(const kc_graph *g, const kc_count_args &a, uint64_t *total, int *overflow) {
    hipStream_t s = g->stream;
    const uint32_t dcap = kc_lds_dcap(g->device, a.k);

    KC_HIP(hipEventRecord(g->ev[0], s));
    // the first count on a handle stages every G+(u) once (timed with the
    // schedule); later counts read it (KC_STAGE_CACHE=0 stages per call instead)
    kc_count_args ac = a;
    const char *sc = getenv("KC_STAGE_CACHE");
    bool staged_now = false;
    if (!(sc && sc[0] == '0')) {
        int wd = kc_tuning_now().wave_dmax;
        wd = wd < 1 ? 1 : (wd > 64 ? 64 : wd);
        kc_graph *gm = const_cast<kc_graph *>(g);
        const int before = gm->staged;
        KC_TRY(kc_stage(gm, wd));
        ac.cached = gm->staged == 1;
        staged_now = before != 1 && gm->staged == 1;
    }
    if (a.sampled && !ac.cached)
        return kc_fail(KC_ENOMEM, "pair sampling counts a masked copy of the staged cache, which is not kept here");
    static const bool biased = getenv("KC_TEST_TOTAL_BIAS") != nullptr;  // the test hook above
    if (staged_now && a.k == 3 && !a.colored && !a.sampled && !a.per_root && !biased) {
        // the staging pass just left q_3 in the result block
        for (int e = 1; e < 8; ++e) KC_HIP(hipEventRecord(g->ev[e], s));
        uint64_t *h_res = kc_pinned_scratch();
        KC_HIP(hipMemcpyAsync(h_res, g->d_res, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        KC_TRY(kc_sync(s));
        float t_sched = 0.f;
        (void)hipEventElapsedTime(&t_sched, g->ev[0], g->ev[1]);
        kc_graph *gm = const_cast<kc_graph *>(g);
        for (int t = 0; t < 3; ++t) gm->t_tier[t] = 0.f;
        stage_tier_times(gm);
        gm->t_schedule = t_sched;
        gm->t_count = 0.f;
        gm->t_total = t_sched;
        *total = h_res[0];
        *overflow = h_res[1] != 0;
        return KC_OK;
    }
    kc_queue q;
    KC_TRY(kc_build_queue(g, a.k, a.policy, dcap, q));
    KC_HIP(hipEventRecord(g->ev[1], s));
    if (a.per_root) KC_HIP(hipMemsetAsync(a.per_root, 0, (size_t)g->n * sizeof(uint64_t), s));
    kc_tmp gscr;
    size_t slice_words = 0;
    uint32_t scratch_blocks = 0;
    KC_TRY(kc_count_scratch(g, q, a.k, gscr, slice_words, scratch_blocks));
    // pair sampling: the count reads a masked copy of the cache through a view of the handle
    kc_tmp mrows, mbits;
    kc_graph view;
    const kc_graph *gc = g;
    if (a.sampled) {
        KC_TRY(kc_tmp_alloc(mrows, (size_t)(g->m ? g->m : 1) * 8, s));
        KC_TRY(kc_tmp_alloc(mbits, (size_t)(g->stage_words ? g->stage_words : 1) * 8, s));
        if (g->m)
            hipLaunchKernelGGL(k_pair_mask_rows, dim3((unsigned)((g->m + 255) / 256)), dim3(256), 0, s,
                               (const uint64_t *)g->optr, (const uint32_t *)g->ocol, (const uint32_t *)g->rank2id, g->n,
                               g->m, (uint32_t)g->stage_wd, (const uint64_t *)g->lrows, mrows.as<uint64_t>(), a.seed,
                               a.pair_t);
        if (g->dq_ready && g->dq_wd == g->stage_wd && g->dq_wide)
            hipLaunchKernelGGL(k_pair_mask_bitmaps, dim3(g->dq_wide), dim3(256), 0, s, (const uint32_t *)g->dq,
                               (const uint64_t *)g->optr, (const uint32_t *)g->ocol, (const uint32_t *)g->rank2id,
                               (const uint64_t *)g->woff, (const uint64_t *)g->wbits, mbits.as<uint64_t>(), a.seed,
                               a.pair_t);
        else if (g->dq_wide || !g->dq_ready)
            return kc_fail(KC_ESTATE, "pair sampling needs the degree queue of the staged cache");
        KC_HIP(hipGetLastError());
        view = *g;
        view.lrows = mrows.as<uint64_t>();
        view.wbits = mbits.as<uint64_t>();
        view.wbits_raw = g->wbits;  // work items were split on the bitmaps as staged
        gc = &view;
    }
    // the second stream (the workgroup tier's large roots beside its small ones) is
    // created on first use, so handles that never split their tier hold none
    const bool side = q.wg_items2 != nullptr;
    if (side && !g->side) {
        kc_graph *gm = const_cast<kc_graph *>(g);
        KC_HIP(hipStreamCreateWithFlags(&gm->side, hipStreamNonBlocking));  // default priority
        KC_HIP(hipEventCreateWithFlags(&gm->fork, hipEventDisableTiming));
        KC_HIP(hipEventCreateWithFlags(&gm->join, hipEventDisableTiming));
        if (gc == &view) {
            view.side = g->side;
            view.fork = g->fork;
            view.join = g->join;
        }
    }
    hipEvent_t tev[6] = {g->ev[2], g->ev[3], g->ev[4], g->ev[5], g->ev[6], g->ev[7]};
    KC_TRY(kc_count_launch(gc, q, ac, g->d_res, nullptr, 0, nullptr, gscr.as<uint64_t>(), slice_words, scratch_blocks,
                           s, tev, side));
    uint64_t *h_res = kc_pinned_scratch();
    KC_HIP(hipMemcpyAsync(h_res, g->d_res, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    KC_TRY(kc_sync(s));
    float t_sched = 0.f, t_count = 0.f, tt[3] = {0.f, 0.f, 0.f};
    (void)hipEventElapsedTime(&t_sched, g->ev[0], g->ev[1]);
    (void)hipEventElapsedTime(&t_count, g->ev[1], g->ev[5]);
    (void)hipEventElapsedTime(&tt[2], g->ev[2], g->ev[3]);
    (void)hipEventElapsedTime(&tt[1], g->ev[3], g->ev[4]);
    (void)hipEventElapsedTime(&tt[0], g->ev[6], g->ev[7]);
    kc_graph *gm = const_cast<kc_graph *>(g);
    for (int t = 0; t < 3; ++t) gm->t_tier[t] = tt[t];
    if (staged_now) stage_tier_times(gm);
    gm->t_schedule = t_sched;
    gm->t_count = t_count;
    gm->t_total = t_sched + t_count;
    *total = h_res[0];
    *overflow = h_res[1] != 0;
    return KC_OK;
}
