// Per-node clique-membership counts.
//
// Section 3 remarks that the round-3 reducer of a root u can report, for every
// node v of its sub-problem, how many of the cliques it found contain v; the
// number of k-cliques that contain v is then the sum of these reports over all
// roots.  Here each root's (k-1)-cliques of G+(u) are counted with attribution:
// u takes all of them, a node of Gamma+(u) the ones it belongs to, and the
// per-node totals are added into a device array indexed by original id.
//
// The local graphs are read from the handle's staged cache (one 64-bit row per
// node of a root with out-degree <= 64, the packed upper-triangular bitmap of a
// larger root).  One wave takes one work item:
//   d <= 64   the whole root: its rows form a one-word local graph;
//   d > 64    a share of the root's first-level nodes (i = part, part + parts, ...).
//             A candidate set of more than 64 nodes that still needs three or more
//             nodes is split one level further, wave-wide, over bitmaps of
//             ceil(d / 64) words kept in LDS; one that needs two (its edges) is
//             taken by the lanes, one member each; one of at most 64 nodes is
//             compacted into a one-word local graph.  The root's nodes are counted
//             in LDS and added to the global array once per item.
// A one-word local graph is counted by the lanes, one edge (i, j) of it per task:
// the candidate set P = row_i & row_j is searched depth-first by the lane, each
// finished clique adds one to every node of it (a node found at the last level
// adds one at once; a node on the path adds the size of its subtree when the lane
// leaves it).  The wide roots' items run first, in a kernel with the LDS they
// need; the one-word roots after them, in one with none.  Global sums are 64-bit
// and carry-checked.
#include "kc_internal.h"

namespace {

static_assert(KC_KMAX <= 10, "32-bit local counters hold C(63, k - 2) for k <= 10 only");

constexpr int PN_WAVES = 4;  // waves per block at most (LDS may allow fewer)
constexpr uint32_t PN_CHUNK = 4;  // work items a wave takes at a time
// first-level nodes per work item of a root with d > 64: at k = 3 the lanes take one
// each; from k = 4 on the wave takes them one after the other
constexpr uint32_t PN_WIDE_SHARE = 16;
constexpr uint32_t PN_WIDE_SHARE3 = 64;

// Depth-first levels a lane keeps: with ell nodes to find in a local graph, an edge
// task leaves ell - 2 to choose in its candidate set, the last of them found
// without a push, so ell - 3 levels; ell <= k - 1.
constexpr int pn_levels(int k) { return k - 4 > 1 ? k - 4 : 1; }

template <int NL>
struct PnArea {
    uint64_t rows[64];     // one-word local graph: bit j of row i iff local j is in Gamma+(local i)
    uint32_t pc[64];       // per-local-node counts of the current local graph (below 2^32:
                           // a node of a 64-node graph is in at most C(63, 8) 9-cliques)
    uint32_t mem[64];      // local node -> its index in Gamma+(u)
    uint32_t pre[64];      // first edge task of each row
    uint64_t st[NL][64];   // per-lane depth-first candidate sets
    uint64_t acc[NL][64];  // per-lane subtree totals of the node taken at each level
    uint8_t nd[NL][64];    // per-lane node taken at each level
    // wave-uniform state of the wide levels (one frame per level)
    uint32_t wpos[KC_KMAX];  // word of the frame's set being scanned
    uint32_t wv[KC_KMAX];    // node the frame descended through
    uint64_t wcur[KC_KMAX];  // bits of that word not taken yet
    uint64_t wacc[KC_KMAX];  // cliques found below the frame
};

struct PnParams {
    const uint64_t *optr;
    const uint32_t *ocol;
    const uint32_t *rank2id;
    const uint64_t *lrows;
    const uint64_t *wbits;
    const uint64_t *woff;
    const uint64_t *items;   // rank << 32 | part << 16 | parts
    const uint64_t *ilo;     // device: first item of this launch (null: 0)
    const uint64_t *ihi;     // device: end of this launch's items
    uint32_t *cursor;        // items of this launch claimed so far
    uint64_t *out;           // per-node counts, by original id
    uint32_t *ovf;           // set when a per-node sum carries out of 64 bits
    uint32_t stage_wd;       // roots up to this out-degree have one-word rows at lrows
    uint32_t wmax;           // words of a wide set: ceil(max out-degree / 64)
    uint32_t lds_rc;         // wide roots count their nodes in LDS (64 * wmax counters per wave)
    size_t wave_words;       // dynamic LDS words per wave: frames, counters, word prefix
};

__device__ __forceinline__ void pn_add(const PnParams &p, uint32_t rank, uint64_t v) {
    if (!v) return;
    uint64_t *dst = p.out + p.rank2id[rank];
    const uint64_t old = atomicAdd((unsigned long long *)dst, (unsigned long long)v);
    if (old + v < old) atomicOr(p.ovf, 1u);
}

// Leaf attribution: every node of P adds one.
template <int NL>
__device__ __forceinline__ void pn_leaf(PnArea<NL> &A, uint64_t P) {
    for (; P; P &= P - 1) atomicAdd(&A.pc[__builtin_ctzll(P)], 1u);
}

// The ell-cliques of the one-word local graph A.rows[0, s) (rows t >= s zero): the
// per-node counts land in A.pc[0, s), the wave-uniform total is returned.
// From ell = 3 on the tasks are the graph's edges (i, j): the R = ell - 2 further
// nodes are chosen depth-first inside P = row_i & row_j by one lane.  Idle lanes
// take new tasks together once at least 16 of them wait (or none is busy), so the
// lanes do not wait for each other's subtrees.  A lane keeps per level the node it
// took and the cliques found below it (added to that node when the lane leaves the
// level), and the task's total (added to i and j when the task ends).
template <int NL>
__device__ uint64_t pn_local(PnArea<NL> &A, uint32_t s, int ell) {
    const uint32_t lane = kc_lane();
    A.pc[lane] = 0;
    kc_wave_sync();
    const uint64_t row = A.rows[lane];
    uint64_t total = 0;
    if (ell <= 0) {
        total = lane == 0 ? 1u : 0u;  // the empty clique: the path above alone
    } else if (ell == 1) {
        if (lane < s) A.pc[lane] = 1;
        total = lane < s ? 1u : 0u;
    } else if (ell == 2) {
        const uint64_t c = (uint64_t)__popcll(row);
        if (c) atomicAdd(&A.pc[lane], (uint32_t)c);
        pn_leaf(A, row);
        total = c;
    } else {
        const int R = ell - 2;
        const uint32_t c = (uint32_t)__popcll(row);
        const uint32_t incl = kc_wave_incl_u32(c);
        const uint32_t E = __shfl(incl, 63, 64);
        A.pre[lane] = incl - c;
        kc_wave_sync();
        int depth = -1;
        uint32_t ti = 0, tj = 0;
        uint64_t tt = 0;  // cliques of the lane's current task
        uint32_t next = 0;
        for (;;) {
            const uint64_t idle = __ballot(depth < 0);
            const uint32_t nidle = (uint32_t)__popcll(idle);
            if (next < E && (nidle >= 16 || nidle == 64)) {
                const uint32_t t = next + (uint32_t)__popcll(idle & kc_lanemask_lt());
                next += nidle;
                if (depth < 0 && t < E) {
                    const uint32_t i = kc_seg_find(A.pre, s, t);
                    const uint64_t ri = A.rows[i];
                    const uint32_t j = kc_select_bit(ri, t - A.pre[i]);
                    const uint64_t P = ri & A.rows[j];
                    if (R == 1) {
                        const uint64_t cc = (uint64_t)__popcll(P);
                        if (cc) {
                            pn_leaf(A, P);
                            atomicAdd(&A.pc[i], (uint32_t)cc);
                            atomicAdd(&A.pc[j], (uint32_t)cc);
                            total += cc;
                        }
                    } else if ((int)__popcll(P) >= R) {
                        depth = 0;
                        A.st[0][lane] = P;
                        ti = i;
                        tj = j;
                        tt = 0;
                    }
                }
            } else if (nidle == 64) {
                break;
            }
            if (depth >= 0) {
                uint64_t cur = A.st[depth][lane];
                if (cur == 0) {
                    // level exhausted: the node its parent level took is done
                    if (depth > 0) {
                        const uint64_t a = A.acc[depth - 1][lane];
                        if (a) atomicAdd(&A.pc[A.nd[depth - 1][lane]], (uint32_t)a);
                        if (depth >= 2) A.acc[depth - 2][lane] += a;
                        else tt += a;
                    } else if (tt) {
                        atomicAdd(&A.pc[ti], (uint32_t)tt);
                        atomicAdd(&A.pc[tj], (uint32_t)tt);
                        total += tt;
                    }
                    --depth;
                } else {
                    const uint32_t v = (uint32_t)__builtin_ctzll(cur);
                    cur &= cur - 1;
                    A.st[depth][lane] = cur;
                    const uint64_t child = cur & A.rows[v];
                    const int rem = R - depth - 1;  // nodes still to choose after v
                    if (rem == 1) {
                        const uint64_t cc = (uint64_t)__popcll(child);
                        if (cc) {
                            atomicAdd(&A.pc[v], (uint32_t)cc);
                            pn_leaf(A, child);
                            if (depth >= 1) A.acc[depth - 1][lane] += cc;
                            else tt += cc;
                        }
                    } else if ((int)__popcll(child) >= rem) {
                        A.nd[depth][lane] = (uint8_t)v;
                        A.acc[depth][lane] = 0;
                        ++depth;
                        A.st[depth][lane] = child;
                    }
                }
            }
        }
    }
    kc_wave_sync();
    return kc_wave_sum_u64(total);
}

// A root with d > 64: its packed bitmap, and where the counts of its nodes go.
// With rc set (a per-wave LDS array of d counters), nodes of Gamma+(u) are counted
// in LDS and added to the global array once per work item; otherwise directly.
struct WideRoot {
    const uint64_t *bm;  // packed upper-triangular bitmap
    uint64_t o;          // start of the root's out-list
    uint32_t W;          // words per row
    uint64_t *rc;        // LDS counters of the root's nodes, or null
    uint32_t *wpre;      // LDS: set bits before each word of a set (W entries)
};

__device__ __forceinline__ void wr_add(const PnParams &p, const WideRoot &R, uint32_t x, uint64_t v) {
    if (!v) return;
    if (R.rc) atomicAdd((unsigned long long *)&R.rc[x], (unsigned long long)v);
    else pn_add(p, p.ocol[R.o + x], v);
}

// The edges inside a wide node set with attribution (ell = 2): each member v adds
// |S & row_v| for the edges it starts, each node of S & row_v one.  Lanes take the
// members, which are found from the word prefix of S; with S null the set is every
// node of the root with an index congruent to part modulo parts (first-level nodes
// of a work item) and row_v is taken whole.  Returns the number of edges.
__device__ uint64_t pn_pairs(const PnParams &p, const WideRoot &R, const uint64_t *S, uint32_t cnt, uint32_t d,
                             uint32_t part, uint32_t parts) {
    const uint32_t lane = kc_lane();
    const uint32_t W = R.W;
    if (S) {
        uint32_t base = 0;
        for (uint32_t w0 = 0; w0 < W; w0 += 64) {
            const uint32_t w = w0 + lane;
            const uint32_t c = w < W ? (uint32_t)__popcll(S[w]) : 0u;
            const uint32_t incl = kc_wave_incl_u32(c);
            if (w < W) R.wpre[w] = base + incl - c;
            base += __shfl(incl, 63, 64);
        }
        kc_wave_sync();
    } else {
        cnt = part < d ? (d - part + parts - 1) / parts : 0u;
    }
    uint64_t total = 0;
    for (uint32_t t = lane; t < cnt; t += 64) {
        uint32_t v;
        if (S) {
            const uint32_t w = kc_seg_find(R.wpre, W, t);
            v = 64u * w + kc_select_bit(S[w], t - R.wpre[w]);
        } else {
            v = part + t * parts;
        }
        const uint32_t fw = (v + 1) >> 6;
        const uint64_t *rv = R.bm + kc_tri_rowoff(v, W);
        uint64_t c = 0;
        for (uint32_t w = fw; w < W; ++w) {
            uint64_t x = rv[w - fw];
            if (S) x &= S[w];
            c += (uint64_t)__popcll(x);
            for (; x; x &= x - 1) wr_add(p, R, 64u * w + (uint32_t)__builtin_ctzll(x), 1);
        }
        wr_add(p, R, v, c);
        total += c;
    }
    kc_wave_sync();
    return kc_wave_sum_u64(total);
}

// The ell-cliques (ell >= 1) inside the wide set S (W words, cnt nodes) with
// attribution to its nodes, for a set that is not split further: every member once
// (ell = 1), the edges (ell = 2), or, with at most 64 nodes, a compacted one-word
// local graph.  Returns the total.
template <int NL>
__device__ uint64_t pn_small(const PnParams &p, PnArea<NL> &A, const WideRoot &R, const uint64_t *S, uint32_t cnt,
                             int ell) {
    const uint32_t lane = kc_lane();
    const uint32_t W = R.W;
    if (ell == 1) {
        for (uint32_t w = lane; w < W; w += 64)
            for (uint64_t x = S[w]; x; x &= x - 1) wr_add(p, R, 64u * w + (uint32_t)__builtin_ctzll(x), 1);
        kc_wave_sync();
        return cnt;
    }
    if (ell == 2) return pn_pairs(p, R, S, cnt, 0, 0, 1);
    // members in order
    uint32_t base = 0;
    for (uint32_t w0 = 0; w0 < W; w0 += 64) {
        const uint32_t w = w0 + lane;
        uint64_t x = w < W ? S[w] : 0ull;
        const uint32_t c = (uint32_t)__popcll(x);
        const uint32_t incl = kc_wave_incl_u32(c);
        uint32_t pos = base + incl - c;
        for (; x; x &= x - 1) A.mem[pos++] = 64u * w + (uint32_t)__builtin_ctzll(x);
        base += __shfl(incl, 63, 64);
    }
    kc_wave_sync();
    // row a of the local graph: bit b (b > a) iff mem[b] is in Gamma+(mem[a]); the
    // members are in order, so row mem[a]'s words are read once each
    uint64_t row = 0;
    if (lane < cnt) {
        const uint32_t v = A.mem[lane];
        const uint32_t fw = (v + 1) >> 6;
        const uint64_t *rv = R.bm + kc_tri_rowoff(v, W);
        uint32_t cw = 0xFFFFFFFFu;
        uint64_t word = 0;
        for (uint32_t b = lane + 1; b < cnt; ++b) {
            const uint32_t y = A.mem[b];
            if ((y >> 6) != cw) {
                cw = y >> 6;
                word = rv[cw - fw];
            }
            row |= ((word >> (y & 63u)) & 1ull) << b;
        }
    }
    A.rows[lane] = row;
    kc_wave_sync();
    const uint64_t t = pn_local(A, cnt, ell);
    if (lane < cnt) wr_add(p, R, A.mem[lane], A.pc[lane]);
    kc_wave_sync();  // the area is reused by the next local graph
    return t;
}

// The ell-cliques (ell >= 1) inside the wide set held at wst[0, W) (cnt nodes), with
// per-node attribution; frame f's set sits at wst + f * W.  A set of more than 64
// nodes with ell >= 3 is scanned node by node (v ascending), each v's candidate set
// S & row_v going one frame deeper unless pn_small takes it; the node a frame
// descended through takes that frame's total when the frame ends.
template <int NL>
__device__ uint64_t pn_wide(const PnParams &p, PnArea<NL> &A, const WideRoot &R, uint64_t *wst, uint32_t cnt,
                            int ell) {
    const uint32_t lane = kc_lane();
    const uint32_t W = R.W;
    if (cnt < (uint32_t)ell) return 0;
    if (cnt <= 64 || ell <= 2) return pn_small(p, A, R, wst, cnt, ell);
    int f = 0;
    if (lane == 0) {
        A.wpos[0] = 0;
        A.wcur[0] = wst[0];
        A.wacc[0] = 0;
    }
    kc_wave_sync();
    for (;;) {
        const uint64_t *S = wst + (size_t)f * W;
        uint32_t pos = A.wpos[f];
        uint64_t cur = A.wcur[f];
        while (cur == 0 && ++pos < W) cur = S[pos];
        if (cur == 0) {
            const uint64_t tot = A.wacc[f];
            kc_wave_sync();
            if (f == 0) return tot;
            --f;
            if (lane == 0) {
                wr_add(p, R, A.wv[f], tot);
                A.wacc[f] += tot;
            }
            kc_wave_sync();
            continue;
        }
        const uint32_t v = 64u * pos + (uint32_t)__builtin_ctzll(cur);
        cur &= cur - 1;
        // the child set S & row_v (row v holds words fw .. W-1) one frame down
        const uint32_t fw = (v + 1) >> 6;
        const uint64_t *rv = R.bm + kc_tri_rowoff(v, W);
        uint64_t *C = wst + (size_t)(f + 1) * W;
        uint32_t c = 0;
        for (uint32_t w = lane; w < W; w += 64) {
            const uint64_t x = w >= fw ? S[w] & rv[w - fw] : 0ull;
            C[w] = x;
            c += (uint32_t)__popcll(x);
        }
        c = kc_wave_sum_u32(c);
        kc_wave_sync();
        if (lane == 0) {
            A.wpos[f] = pos;
            A.wcur[f] = cur;
        }
        const int ellc = ell - f - 1;  // clique size left for the child
        if (c < (uint32_t)ellc) {
            kc_wave_sync();
            continue;
        }
        if (c <= 64 || ellc <= 2) {
            const uint64_t t = pn_small(p, A, R, C, c, ellc);
            if (lane == 0) {
                wr_add(p, R, v, t);
                A.wacc[f] += t;
            }
            kc_wave_sync();
            continue;
        }
        if (lane == 0) {
            A.wv[f] = v;
            A.wpos[f + 1] = 0;
            A.wcur[f + 1] = C[0];
            A.wacc[f + 1] = 0;
        }
        ++f;
        kc_wave_sync();
    }
}

// One work item.  WIDE: the kernel that takes the roots above the one-wave limit of
// the staged cache (with the LDS for wide roots); otherwise every root has d <= 64.
template <int NL, bool WIDE>
__device__ void pn_item(const PnParams &p, PnArea<NL> &A, uint64_t *wdyn, int ell, uint32_t r, uint32_t part,
                        uint32_t parts) {
    const uint32_t lane = kc_lane();
    const uint64_t o = p.optr[r];
    const uint32_t d = (uint32_t)(p.optr[r + 1] - o);
    if (!WIDE || d <= 64) {
        const uint64_t *src = d <= p.stage_wd ? p.lrows + o : p.wbits + p.woff[r];
        A.rows[lane] = lane < d ? src[lane] : 0ull;
        A.mem[lane] = lane;
        kc_wave_sync();
        const uint64_t t = pn_local(A, d, ell);
        if (lane < d) pn_add(p, p.ocol[o + lane], A.pc[lane]);
        if (lane == 0) pn_add(p, r, t);
        kc_wave_sync();
        return;
    }
    if constexpr (!WIDE) return;
    WideRoot R;
    R.bm = p.wbits + p.woff[r];
    R.o = o;
    R.W = (d + 63) >> 6;
    uint64_t *wst = wdyn;  // ell - 1 frames of wmax words
    R.rc = p.lds_rc ? wdyn + (size_t)(ell - 1) * p.wmax : nullptr;
    R.wpre = (uint32_t *)(wdyn + (size_t)(ell - 1) * p.wmax + (p.lds_rc ? 64ull * p.wmax : 0ull));
    if (R.rc) {
        for (uint32_t x = lane; x < d; x += 64) R.rc[x] = 0;
        kc_wave_sync();
    }
    uint64_t root_total = 0;
    if (ell == 2) {
        root_total = pn_pairs(p, R, nullptr, 0, d, part, parts);
    } else {
        for (uint32_t i = part; i < d; i += parts) {
            // frame 0: row i, the candidate set of first-level node i
            const uint32_t fw = (i + 1) >> 6;
            const uint64_t *ri = R.bm + kc_tri_rowoff(i, R.W);
            uint32_t c = 0;
            for (uint32_t w = lane; w < R.W; w += 64) {
                const uint64_t x = w >= fw ? ri[w - fw] : 0ull;
                wst[w] = x;
                c += (uint32_t)__popcll(x);
            }
            c = kc_wave_sum_u32(c);
            kc_wave_sync();
            const uint64_t t = pn_wide(p, A, R, wst, c, ell - 1);
            if (lane == 0) wr_add(p, R, i, t);
            kc_wave_sync();
            root_total += t;
        }
    }
    if (R.rc) {
        for (uint32_t x = lane; x < d; x += 64) pn_add(p, p.ocol[o + x], R.rc[x]);
        kc_wave_sync();
    }
    if (lane == 0) pn_add(p, r, root_total);
}

template <int K, bool WIDE>
__global__ void __launch_bounds__(PN_WAVES * 64) k_per_node(PnParams p) {
    constexpr int NL = pn_levels(K);
    __shared__ PnArea<NL> areas[PN_WAVES];
    extern __shared__ uint64_t pn_dyn[];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    PnArea<NL> &A = areas[wave];
    uint64_t *wdyn = pn_dyn + (size_t)wave * p.wave_words;
    const uint64_t lo = p.ilo ? *p.ilo : 0ull, count = *p.ihi - lo;
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(p.cursor, PN_CHUNK);
        it = (uint32_t)__builtin_amdgcn_readfirstlane((int)it);
        if (it >= count) break;
        const uint32_t end = (uint64_t)it + PN_CHUNK < count ? it + PN_CHUNK : (uint32_t)count;
        for (; it < end; ++it) {
            const uint64_t item = p.items[lo + it];
            pn_item<NL, WIDE>(p, A, wdyn, K - 1, (uint32_t)(item >> 32), (uint32_t)(item >> 16) & 0xFFFFu,
                              (uint32_t)item & 0xFFFFu);
        }
    }
}

// work items per queue position: none below k - 1 out-neighbours, one for a root
// with d <= 64, ceil(d / share) for a larger one
__global__ void k_pn_parts(const uint32_t *dq, uint32_t nq, const uint64_t *optr, uint32_t dmin, uint32_t share,
                           uint64_t *parts) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const uint32_t r = dq[i];
    const uint64_t d = optr[r + 1] - optr[r];
    uint64_t c = d < dmin ? 0 : (d <= 64 ? 1 : (d + share - 1) / share);
    parts[i] = c > 0xFFFF ? 0xFFFF : c;
}

__global__ void k_pn_emit(const uint32_t *dq, uint32_t nq, const uint64_t *parts, const uint64_t *first,
                          uint64_t *items) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const uint64_t c = parts[i], b = first[i], r = dq[i];
    for (uint64_t t = 0; t < c; ++t) items[b + t] = r << 32 | t << 16 | c;
}

__global__ void k_pn_fill(uint64_t *out, uint32_t n, uint64_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

// k = 2: the degree of every node (its out-degree plus the edges that point at it)
__global__ void k_pn_degree(const uint64_t *optr, const uint32_t *ocol, const uint32_t *rank2id, uint32_t n,
                            uint64_t *out) {
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint64_t b = optr[r], e = optr[r + 1];
    atomicAdd((unsigned long long *)&out[rank2id[r]], (unsigned long long)(e - b));
    for (uint64_t x = b; x < e; ++x) atomicAdd((unsigned long long *)&out[rank2id[ocol[x]]], 1ull);
}

// The wide roots' items (the dq's first part) with the LDS for wide roots, then the
// rest with none, so that the one-word roots run at full occupancy.
template <int K>
kc_status pn_launch(PnParams p, const uint64_t *split, uint32_t *cursors, size_t lds_max, int cus, hipStream_t s) {
    const size_t stat = sizeof(PnArea<pn_levels(K)>) * PN_WAVES;
    // per wave: K - 2 frames of wmax words, then (when they fit) 64 * wmax node
    // counters, then the word prefix (wmax 32-bit entries)
    const size_t frames = (size_t)(K - 2) * p.wmax, pre = (p.wmax + 1) / 2;
    auto fits = [&](int nw, size_t words) { return stat + (size_t)nw * words * 8 <= lds_max; };
    int nw = PN_WAVES;
    p.lds_rc = 1;
    p.wave_words = frames + 64ull * p.wmax + pre;
    while (nw > 1 && !fits(nw, p.wave_words)) nw /= 2;
    if (!fits(nw, p.wave_words)) {
        p.lds_rc = 0;
        p.wave_words = frames + pre;
        nw = PN_WAVES;
        while (nw > 1 && !fits(nw, p.wave_words)) nw /= 2;
        if (!fits(nw, p.wave_words))
            return kc_fail(KC_EINVAL, "out-degree %u needs %zu bytes of LDS per wave for per-node counts at k=%d",
                           p.wmax * 64, p.wave_words * 8, K);
    }
    const void *fw = (const void *)&k_per_node<K, true>;
    const size_t dyn = (size_t)nw * p.wave_words * 8;
    (void)hipFuncSetAttribute(fw, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(lds_max - stat));
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fw, nw * 64, dyn) != hipSuccess || occ < 1) occ = 1;
    const uint64_t *end = p.ihi;
    p.ilo = nullptr;
    p.ihi = split;
    p.cursor = cursors;
    hipLaunchKernelGGL((k_per_node<K, true>), dim3((unsigned)(cus * occ)), dim3(nw * 64), dyn, s, p);
    KC_HIP(hipGetLastError());
    const void *fn = (const void *)&k_per_node<K, false>;
    occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, PN_WAVES * 64, 0) != hipSuccess || occ < 1) occ = 1;
    p.ilo = split;
    p.ihi = end;
    p.cursor = cursors + 1;
    p.wave_words = 0;
    hipLaunchKernelGGL((k_per_node<K, false>), dim3((unsigned)(cus * occ)), dim3(PN_WAVES * 64), 0, s, p);
    KC_HIP(hipGetLastError());
    return KC_OK;
}

inline unsigned grid256(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" kc_status kc_count_per_node(const kc_graph *g, int32_t k, uint64_t *dev_counts) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (!dev_counts) return kc_fail(KC_EINVAL, "dev_counts is NULL");
    if (k < 1 || k > KC_KMAX) return kc_fail(KC_EINVAL, "k=%d outside [1, %d]", k, KC_KMAX);
    if (!g->oriented) return kc_fail(KC_ESTATE, "kc_orient has not been called");
    hipStream_t s = g->stream;
    const uint32_t n = g->n;
    if (n == 0) return KC_OK;
    hipLaunchKernelGGL(k_pn_fill, dim3(grid256(n)), dim3(256), 0, s, dev_counts, n, k == 1 ? 1ull : 0ull);
    KC_HIP(hipGetLastError());
    if (k == 2)
        hipLaunchKernelGGL(k_pn_degree, dim3(grid256(n)), dim3(256), 0, s, (const uint64_t *)g->optr,
                           (const uint32_t *)g->ocol, (const uint32_t *)g->rank2id, n, dev_counts);
    KC_HIP(hipGetLastError());
    if (k <= 2) return kc_sync(s);

    // the staged cache holds every root's local graph
    kc_graph *gm = const_cast<kc_graph *>(g);
    int wd = kc_tuning_now().wave_dmax;
    wd = wd < 1 ? 1 : (wd > 64 ? 64 : wd);
    KC_TRY(kc_stage(gm, wd));
    if (gm->staged != 1)
        return kc_fail(KC_ENOMEM, "per-node counts read the staged G+(u) cache, which is not kept here");
    kc_queue q;
    KC_TRY(kc_build_queue(g, 3, KC_SCHED_DEGREE, kc_lds_dcap(g->device, 3), q));
    if (!g->dq_ready) return kc_fail(KC_ESTATE, "degree queue not built");
    const uint32_t nq = g->dq_wide + g->dq_narrow;  // roots with out-degree >= 2, widest first
    if (nq == 0) return kc_sync(s);

    kc_tmp parts, first, items, ctr;
    KC_TRY(kc_tmp_alloc(parts, (size_t)nq * 8, s));
    KC_TRY(kc_tmp_alloc(first, ((size_t)nq + 1) * 8, s));
    const size_t max_items = (size_t)nq + (size_t)(g->m / PN_WIDE_SHARE) + g->dq_wide + 1;
    KC_TRY(kc_tmp_alloc(items, max_items * 8, s));
    KC_TRY(kc_tmp_alloc(ctr, 16, s));
    hipLaunchKernelGGL(k_pn_parts, dim3(grid256(nq)), dim3(256), 0, s, (const uint32_t *)g->dq, nq,
                       (const uint64_t *)g->optr, (uint32_t)(k - 1), k == 3 ? PN_WIDE_SHARE3 : PN_WIDE_SHARE,
                       parts.as<uint64_t>());
    KC_HIP(hipGetLastError());
    KC_TRY(kc_scan_excl_u64(parts.as<uint64_t>(), first.as<uint64_t>(), nq, first.as<uint64_t>() + nq, s));
    hipLaunchKernelGGL(k_pn_emit, dim3(grid256(nq)), dim3(256), 0, s, (const uint32_t *)g->dq, nq,
                       (const uint64_t *)parts.as<uint64_t>(), (const uint64_t *)first.as<uint64_t>(),
                       items.as<uint64_t>());
    KC_HIP(hipGetLastError());
    KC_HIP(hipMemsetAsync(ctr.p, 0, 16, s));  // two launch cursors and the overflow flag

    PnParams p;
    p.optr = g->optr;
    p.ocol = g->ocol;
    p.rank2id = g->rank2id;
    p.lrows = g->lrows;
    p.wbits = g->wbits;
    p.woff = g->woff;
    p.items = items.as<uint64_t>();
    p.ilo = nullptr;
    p.ihi = first.as<uint64_t>() + nq;
    p.cursor = nullptr;
    p.out = dev_counts;
    p.ovf = ctr.as<uint32_t>() + 2;
    p.stage_wd = (uint32_t)g->stage_wd;
    p.wmax = (g->max_outdeg + 63) / 64;
    if (p.wmax == 0) p.wmax = 1;
    int cus = 0, lds = 0;
    KC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
    KC_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device));
    if (cus <= 0) cus = 1;
    const size_t lds_max = lds > 0 ? (size_t)lds : 65536;
    const uint64_t *split = first.as<uint64_t>() + g->dq_wide;  // first item of the one-word roots
    switch (k) {
    case 3: KC_TRY(pn_launch<3>(p, split, ctr.as<uint32_t>(), lds_max, cus, s)); break;
    case 4: KC_TRY(pn_launch<4>(p, split, ctr.as<uint32_t>(), lds_max, cus, s)); break;
    case 5: KC_TRY(pn_launch<5>(p, split, ctr.as<uint32_t>(), lds_max, cus, s)); break;
    case 6: KC_TRY(pn_launch<6>(p, split, ctr.as<uint32_t>(), lds_max, cus, s)); break;
    case 7: KC_TRY(pn_launch<7>(p, split, ctr.as<uint32_t>(), lds_max, cus, s)); break;
    case 8: KC_TRY(pn_launch<8>(p, split, ctr.as<uint32_t>(), lds_max, cus, s)); break;
    case 9: KC_TRY(pn_launch<9>(p, split, ctr.as<uint32_t>(), lds_max, cus, s)); break;
    case 10: KC_TRY(pn_launch<10>(p, split, ctr.as<uint32_t>(), lds_max, cus, s)); break;
    default: return kc_fail(KC_EINVAL, "k=%d", k);
    }
    uint32_t *h = (uint32_t *)kc_pinned_scratch();
    KC_HIP(hipMemcpyAsync(h, ctr.as<uint32_t>() + 2, 4, hipMemcpyDeviceToHost, s));
    KC_TRY(kc_sync(s));
    if (h[0]) return kc_fail(KC_EOVERFLOW, "a per-node count at k=%d needs more than 64 bits", k);
    return KC_OK;
}
