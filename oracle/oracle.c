/*
 * CPU ORACLE for k-clique counting.  TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow and meant to be checked by eye against the paper (Finocchi,
 * Finocchi & Fusco, "Clique counting in MapReduce: theory and experiments").
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
 * it.  It shares no code, header, table or helper with the GPU library.
 *
 * What it computes, and where the paper defines it:
 *   - q_k, the number of k-node cliques (Section 2, notation).
 *   - The total order:  x < y  iff  d(x) < d(y), or d(x) = d(y) and x < y, with
 *     d the degree in the simple graph and x, y the original labels (Section 2).
 *     Written here as key(x) = (d(x) << 32) | x compared as an unsigned integer.
 *   - The high-neighbourhood Gamma+(u) = { x in Gamma(u) : u < x } (Section 2).
 *   - Exact counting (Section 3, Algorithm 1, Theorem 1): every clique is counted
 *     once, by its smallest node u, as a (k-1)-clique of the subgraph induced by
 *     Gamma+(u).  The local count uses neighbourhood intersection:
 *         cnt(P, 1) = |P|,   cnt(P, l) = sum_{v in P} cnt(P n Gamma+(v), l - 1).
 *   - Colour sampling cFFF_k (Section 6, colour-based sampling): the nodes of each
 *     Gamma+(u) are coloured independently per root u with c colours and only
 *     monochromatic pairs are kept; the raw count is scaled by c^(k-2).  The
 *     global variant colours every node once (the Pagh-Tsourakakis colouring the
 *     paper builds on) and keeps k-cliques whose k nodes share one colour; its
 *     scale is c^(k-1).
 *   - Per-root intersection work (the paper instruments sub-problem sizes,
 *     Section 4): W(u, k) = sum_{l=1}^{k-2} c_l(G+(u)).
 *   - Per-node clique-membership counts (Section 3, the remark after the round-3
 *     reducers): the k-cliques containing each node, as the sum over roots of the
 *     cliques of G+(u) that contain it, and by the plain definition.
 *
 * Colour hash (the paper leaves the colouring's randomness unspecified; this is
 * the reading used): SplitMix64's finaliser mix64 (Steele, Lea & Flood 2014),
 *   H(seed, u, x) = mix64(seed ^ mix64((u << 32) | x)),  H(seed, x) = mix64(seed ^ mix64(x)),
 *   colour(h, c) = ((h >> 32) * c) >> 32.
 *
 * Every 64-bit sum is overflow-checked; overflow is reported as status -4.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { KCO_OK = 0, KCO_EINVAL = -1, KCO_ENOMEM = -3, KCO_EOVERFLOW = -4 };
enum { KCO_COLOR_PER_ROOT = 0, KCO_COLOR_GLOBAL = 1 };

typedef struct kco_graph {
    uint32_t n;
    uint64_t m;          /* undirected edges of the simple graph */
    uint32_t *eu, *ev;   /* canonical edges, eu[i] < ev[i], sorted */
    uint32_t *deg;       /* d(x) in the simple graph */
    uint64_t *hp;        /* Gamma+ lists, original ids: hn[hp[u] .. hp[u+1]) */
    uint32_t *hn;        /* each list sorted by the total order */
    uint32_t *rank2id;   /* nodes sorted by the total order */
    uint32_t *rank;      /* position of each node in that order */
} kco_graph;

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* key(x) = (d(x), x): the paper's total order as one unsigned integer */
static inline uint64_t key_of(const kco_graph *g, uint32_t x) {
    return ((uint64_t)g->deg[x] << 32) | x;
}

void kco_destroy(kco_graph *g) {
    if (!g) return;
    free(g->eu); free(g->ev); free(g->deg); free(g->hp); free(g->hn);
    free(g->rank2id); free(g->rank);
    free(g);
}

/* Build the simple graph, the degrees, the order and the high-neighbourhoods. */
int kco_create(const uint32_t *src, const uint32_t *dst, uint64_t m_in, uint32_t n, kco_graph **out) {
    if (!out || (m_in && (!src || !dst))) return KCO_EINVAL;
    *out = NULL;
    for (uint64_t i = 0; i < m_in; ++i)
        if (src[i] >= n || dst[i] >= n) return KCO_EINVAL;

    kco_graph *g = (kco_graph *)calloc(1, sizeof(kco_graph));
    if (!g) return KCO_ENOMEM;
    g->n = n;

    /* undirected pairs {min, max}, self-loops dropped, then sorted and deduplicated */
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (m_in ? m_in : 1));
    if (!keys) { kco_destroy(g); return KCO_ENOMEM; }
    uint64_t nk = 0;
    for (uint64_t i = 0; i < m_in; ++i) {
        uint32_t a = src[i], b = dst[i];
        if (a == b) continue;
        uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
        keys[nk++] = ((uint64_t)lo << 32) | hi;
    }
    qsort(keys, nk, sizeof(uint64_t), cmp_u64);
    uint64_t m = 0;
    for (uint64_t i = 0; i < nk; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
    g->m = m;
    g->eu = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
    g->ev = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
    g->deg = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    if (!g->eu || !g->ev || !g->deg) { free(keys); kco_destroy(g); return KCO_ENOMEM; }
    for (uint64_t i = 0; i < m; ++i) {
        g->eu[i] = (uint32_t)(keys[i] >> 32);
        g->ev[i] = (uint32_t)keys[i];
        g->deg[g->eu[i]]++;
        g->deg[g->ev[i]]++;
    }
    free(keys);

    /* the total order over all nodes */
    uint64_t *nk2 = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    g->rank2id = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    g->rank = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!nk2 || !g->rank2id || !g->rank) { free(nk2); kco_destroy(g); return KCO_ENOMEM; }
    for (uint32_t x = 0; x < n; ++x) nk2[x] = key_of(g, x);
    qsort(nk2, n, sizeof(uint64_t), cmp_u64);
    for (uint32_t r = 0; r < n; ++r) {
        g->rank2id[r] = (uint32_t)nk2[r];
        g->rank[g->rank2id[r]] = r;
    }
    free(nk2);

    /* Gamma+(u): each edge goes to its smaller endpoint's list */
    g->hp = (uint64_t *)calloc((uint64_t)n + 1, sizeof(uint64_t));
    g->hn = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
    if (!g->hp || !g->hn) { kco_destroy(g); return KCO_ENOMEM; }
    for (uint64_t i = 0; i < m; ++i) {
        uint32_t a = g->eu[i], b = g->ev[i];
        uint32_t low = key_of(g, a) < key_of(g, b) ? a : b;
        g->hp[low + 1]++;
    }
    for (uint32_t x = 0; x < n; ++x) g->hp[x + 1] += g->hp[x];
    uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * ((uint64_t)n + 1));
    uint64_t *lk = (uint64_t *)malloc(sizeof(uint64_t) * (m ? m : 1));
    if (!fill || !lk) { free(fill); free(lk); kco_destroy(g); return KCO_ENOMEM; }
    memcpy(fill, g->hp, sizeof(uint64_t) * ((uint64_t)n + 1));
    for (uint64_t i = 0; i < m; ++i) {
        uint32_t a = g->eu[i], b = g->ev[i];
        int a_low = key_of(g, a) < key_of(g, b);
        uint32_t low = a_low ? a : b, high = a_low ? b : a;
        lk[fill[low]++] = key_of(g, high);
    }
    for (uint32_t x = 0; x < n; ++x) {
        uint64_t lo = g->hp[x], hi = g->hp[x + 1];
        qsort(lk + lo, hi - lo, sizeof(uint64_t), cmp_u64);
        for (uint64_t j = lo; j < hi; ++j) g->hn[j] = (uint32_t)lk[j];
    }
    free(fill);
    free(lk);
    *out = g;
    return KCO_OK;
}

uint32_t kco_n(const kco_graph *g) { return g->n; }
uint64_t kco_m(const kco_graph *g) { return g->m; }

void kco_canon_edges(const kco_graph *g, uint32_t *eu, uint32_t *ev) {
    memcpy(eu, g->eu, sizeof(uint32_t) * g->m);
    memcpy(ev, g->ev, sizeof(uint32_t) * g->m);
}
void kco_degrees(const kco_graph *g, uint32_t *deg) { memcpy(deg, g->deg, sizeof(uint32_t) * g->n); }
void kco_rank2id(const kco_graph *g, uint32_t *r2i) { memcpy(r2i, g->rank2id, sizeof(uint32_t) * g->n); }

/* Gamma+ lists as given (original ids, sorted by the order). */
void kco_high_csr(const kco_graph *g, uint64_t *hp, uint32_t *hn) {
    memcpy(hp, g->hp, sizeof(uint64_t) * ((uint64_t)g->n + 1));
    memcpy(hn, g->hn, sizeof(uint32_t) * g->m);
}

/* The same lists relabelled by position in the order: row r is node rank2id[r]. */
void kco_rank_csr(const kco_graph *g, uint64_t *optr, uint32_t *ocol) {
    uint64_t pos = 0;
    optr[0] = 0;
    for (uint32_t r = 0; r < g->n; ++r) {
        uint32_t u = g->rank2id[r];
        for (uint64_t j = g->hp[u]; j < g->hp[u + 1]; ++j) ocol[pos++] = g->rank[g->hn[j]];
        optr[r + 1] = pos;
    }
}

uint32_t kco_max_outdeg(const kco_graph *g) {
    uint32_t best = 0;
    for (uint32_t x = 0; x < g->n; ++x) {
        uint64_t d = g->hp[x + 1] - g->hp[x];
        if (d > best) best = (uint32_t)d;
    }
    return best;
}

/* ------------------------------------------------------------------------- */
/* P n Gamma+(v), both sorted by the order: a plain merge. */
static uint64_t intersect(const kco_graph *g, const uint32_t *P, uint64_t np, uint32_t v, uint32_t *out) {
    const uint32_t *N = g->hn + g->hp[v];
    uint64_t nn = g->hp[v + 1] - g->hp[v], i = 0, j = 0, c = 0;
    while (i < np && j < nn) {
        uint64_t a = key_of(g, P[i]), b = key_of(g, N[j]);
        if (a < b) ++i;
        else if (b < a) ++j;
        else { out[c++] = P[i]; ++i; ++j; }
    }
    return c;
}

/* cnt(P, l): the number of l-cliques inside the node set P (P sorted by the
 * order), by neighbourhood intersection.  buf holds l * np entries. */
static int cnt(const kco_graph *g, const uint32_t *P, uint64_t np, int l, uint32_t *buf, uint64_t *out) {
    if (l <= 0) { *out = 1; return KCO_OK; }
    if (l == 1) { *out = np; return KCO_OK; }
    uint64_t total = 0;
    for (uint64_t i = 0; i < np; ++i) {
        uint64_t nq = intersect(g, P, np, P[i], buf);
        uint64_t sub;
        int st = cnt(g, buf, nq, l - 1, buf + np, &sub);
        if (st) return st;
        if (__builtin_add_overflow(total, sub, &total)) return KCO_EOVERFLOW;
    }
    *out = total;
    return KCO_OK;
}

/* q_{u,k-1}: the (k-1)-cliques of G+(u), i.e. the k-cliques whose smallest node is u. */
int kco_count_root(const kco_graph *g, uint32_t u, int k, uint64_t *out) {
    if (!g || !out || u >= g->n || k < 1) return KCO_EINVAL;
    uint64_t d = g->hp[u + 1] - g->hp[u];
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * ((uint64_t)k * d + 1));
    if (!buf) return KCO_ENOMEM;
    int st = cnt(g, g->hn + g->hp[u], d, k - 1, buf, out);
    free(buf);
    return st;
}

/* q_{u,k-1} for a list of roots (original ids). */
int kco_count_roots(const kco_graph *g, int k, const uint32_t *roots, uint64_t nroots, int threads, uint64_t *out) {
    if (!g || k < 1 || (nroots && (!roots || !out))) return KCO_EINVAL;
    for (uint64_t i = 0; i < nroots; ++i) if (roots[i] >= g->n) return KCO_EINVAL;
    int status = KCO_OK;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
    #pragma omp parallel for schedule(dynamic, 16) num_threads(threads)
#endif
    for (int64_t i = 0; i < (int64_t)nroots; ++i) {
        int st = kco_count_root(g, roots[i], k, &out[i]);
        if (st) {
            #pragma omp critical
            status = st;
        }
    }
    (void)threads;
    return status;
}

/* Per-root counts for every node, indexed by original id. */
int kco_count_per_root(const kco_graph *g, int k, int threads, uint64_t *counts) {
    if (!g || !counts || k < 1) return KCO_EINVAL;
    uint32_t *all = (uint32_t *)malloc(sizeof(uint32_t) * (g->n ? g->n : 1));
    if (!all) return KCO_ENOMEM;
    for (uint32_t x = 0; x < g->n; ++x) all[x] = x;
    int st = kco_count_roots(g, k, all, g->n, threads, counts);
    free(all);
    return st;
}

/* q_k = sum over roots of q_{u,k-1}. */
int kco_count(const kco_graph *g, int k, int threads, uint64_t *q) {
    if (!g || !q || k < 1) return KCO_EINVAL;
    uint64_t *c = (uint64_t *)malloc(sizeof(uint64_t) * (g->n ? g->n : 1));
    if (!c) return KCO_ENOMEM;
    int st = kco_count_per_root(g, k, threads, c);
    uint64_t total = 0;
    for (uint32_t x = 0; st == KCO_OK && x < g->n; ++x)
        if (__builtin_add_overflow(total, c[x], &total)) st = KCO_EOVERFLOW;
    free(c);
    if (st == KCO_OK) *q = total;
    return st;
}

/* ------------------------------------------------------------------------- */
/* Colour hash. */
uint64_t kco_mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
uint64_t kco_hash_root(uint64_t seed, uint32_t u, uint32_t x) {
    return kco_mix64(seed ^ kco_mix64(((uint64_t)u << 32) | x));
}
uint64_t kco_hash_node(uint64_t seed, uint32_t x) { return kco_mix64(seed ^ kco_mix64((uint64_t)x)); }
uint32_t kco_color(uint64_t h, uint32_t c) { return (uint32_t)(((h >> 32) * (uint64_t)c) >> 32); }

/* Raw colour-sampled count for one root.
 * Per-root scheme: colour Gamma+(u) with colour(H(seed,u,x), c); each colour
 *   class P_g keeps only its monochromatic pairs, so the root contributes
 *   sum_g cnt(P_g, k-1).
 * Global scheme: colour every node with colour(H(seed,x), c); the root
 *   contributes cnt({x in Gamma+(u) : col(x) = col(u)}, k-1). */
int kco_count_colored_root(const kco_graph *g, uint32_t u, int k, uint32_t c, uint64_t seed, int scheme,
                           uint64_t *out) {
    if (!g || !out || u >= g->n || k < 1 || c == 0) return KCO_EINVAL;
    if (scheme != KCO_COLOR_PER_ROOT && scheme != KCO_COLOR_GLOBAL) return KCO_EINVAL;
    const uint32_t *N = g->hn + g->hp[u];
    uint64_t d = g->hp[u + 1] - g->hp[u];
    uint32_t *col = (uint32_t *)malloc(sizeof(uint32_t) * (d + 1));
    uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * (d + 1));
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * ((uint64_t)k * d + 1));
    if (!col || !P || !buf) { free(col); free(P); free(buf); return KCO_ENOMEM; }
    int st = KCO_OK;
    uint64_t total = 0;
    if (scheme == KCO_COLOR_PER_ROOT) {
        for (uint64_t i = 0; i < d; ++i) col[i] = kco_color(kco_hash_root(seed, u, N[i]), c);
        /* one class per distinct colour present, in order of first appearance */
        for (uint64_t i = 0; i < d && st == KCO_OK; ++i) {
            int seen = 0;
            for (uint64_t j = 0; j < i; ++j) if (col[j] == col[i]) { seen = 1; break; }
            if (seen) continue;
            uint64_t np = 0;
            for (uint64_t j = 0; j < d; ++j) if (col[j] == col[i]) P[np++] = N[j];
            uint64_t sub;
            st = cnt(g, P, np, k - 1, buf, &sub);
            if (st == KCO_OK && __builtin_add_overflow(total, sub, &total)) st = KCO_EOVERFLOW;
        }
    } else {
        uint32_t cu = kco_color(kco_hash_node(seed, u), c);
        uint64_t np = 0;
        for (uint64_t j = 0; j < d; ++j)
            if (kco_color(kco_hash_node(seed, N[j]), c) == cu) P[np++] = N[j];
        st = cnt(g, P, np, k - 1, buf, &total);
    }
    free(col); free(P); free(buf);
    if (st == KCO_OK) *out = total;
    return st;
}

int kco_count_colored_per_root(const kco_graph *g, int k, uint32_t c, uint64_t seed, int scheme, int threads,
                               uint64_t *counts) {
    if (!g || !counts || k < 1 || c == 0) return KCO_EINVAL;
    int status = KCO_OK;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
    #pragma omp parallel for schedule(dynamic, 16) num_threads(threads)
#endif
    for (int64_t x = 0; x < (int64_t)g->n; ++x) {
        int st = kco_count_colored_root(g, (uint32_t)x, k, c, seed, scheme, &counts[x]);
        if (st) {
            #pragma omp critical
            status = st;
        }
    }
    (void)threads;
    return status;
}

int kco_count_colored(const kco_graph *g, int k, uint32_t c, uint64_t seed, int scheme, int threads,
                      uint64_t *raw) {
    if (!g || !raw) return KCO_EINVAL;
    uint64_t *cc = (uint64_t *)malloc(sizeof(uint64_t) * (g->n ? g->n : 1));
    if (!cc) return KCO_ENOMEM;
    int st = kco_count_colored_per_root(g, k, c, seed, scheme, threads, cc);
    uint64_t total = 0;
    for (uint32_t x = 0; st == KCO_OK && x < g->n; ++x)
        if (__builtin_add_overflow(total, cc[x], &total)) st = KCO_EOVERFLOW;
    free(cc);
    if (st == KCO_OK) *raw = total;
    return st;
}

/* ------------------------------------------------------------------------- */
/* Plain pair sampling FFF_k(p) (Section 6, plain pair sampling): every pair of
 * high-neighbours of u that is an edge of G+(u) is kept independently with
 * probability p, and the root contributes the (k-1)-cliques of the sampled G+(u);
 * a k-clique survives when all C(k-1, 2) pairs of its non-minimum nodes do.
 * Randomness (the paper leaves it unspecified): the pair (x, y), x before y in the
 * order, is kept iff (H2 >> 32) < t, with H2 = mix64(H(seed, u, x) ^ mix64(y)) and
 * t = floor(p * 2^32) (t = 2^32 keeps every pair). */
uint64_t kco_hash_pair(uint64_t seed, uint32_t u, uint32_t x, uint32_t y) {
    return kco_mix64(kco_hash_root(seed, u, x) ^ kco_mix64((uint64_t)y));
}

/* l-cliques inside the local node list P (ascending local indices) of a graph
 * given by its upper adjacency matrix adj[i * d + j] (i < j). */
static int pcnt(const uint8_t *adj, uint64_t d, const uint32_t *P, uint64_t np, int l, uint32_t *buf,
                uint64_t *out) {
    if (l <= 0) { *out = 1; return KCO_OK; }
    if (l == 1) { *out = np; return KCO_OK; }
    uint64_t total = 0;
    for (uint64_t a = 0; a < np; ++a) {
        uint64_t nq = 0;
        for (uint64_t b = a + 1; b < np; ++b)
            if (adj[(uint64_t)P[a] * d + P[b]]) buf[nq++] = P[b];
        uint64_t sub;
        int st = pcnt(adj, d, buf, nq, l - 1, buf + np, &sub);
        if (st) return st;
        if (__builtin_add_overflow(total, sub, &total)) return KCO_EOVERFLOW;
    }
    *out = total;
    return KCO_OK;
}

int kco_count_pair_sampled_root(const kco_graph *g, uint32_t u, int k, uint64_t t, uint64_t seed, uint64_t *out) {
    if (!g || !out || u >= g->n || k < 3) return KCO_EINVAL;
    const uint32_t *N = g->hn + g->hp[u];
    const uint64_t d = g->hp[u + 1] - g->hp[u];
    if (d < (uint64_t)(k - 1)) { *out = 0; return KCO_OK; }
    uint8_t *adj = (uint8_t *)calloc(d * d, 1);
    uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * (d * (uint64_t)k + 1));
    if (!adj || !P) { free(adj); free(P); return KCO_ENOMEM; }
    for (uint64_t i = 0; i < d; ++i) {
        /* members of Gamma+(N[i]) that are later members of Gamma+(u): a merge by key */
        const uint32_t *M = g->hn + g->hp[N[i]];
        const uint64_t mm = g->hp[N[i] + 1] - g->hp[N[i]];
        uint64_t a = i + 1, b = 0;
        while (a < d && b < mm) {
            const uint64_t ka = key_of(g, N[a]), kb = key_of(g, M[b]);
            if (ka < kb) ++a;
            else if (kb < ka) ++b;
            else {
                if ((kco_hash_pair(seed, u, N[i], N[a]) >> 32) < t) adj[i * d + a] = 1;
                ++a;
                ++b;
            }
        }
    }
    for (uint64_t i = 0; i < d; ++i) P[i] = (uint32_t)i;
    int st = pcnt(adj, d, P, d, k - 1, P + d, out);
    free(adj);
    free(P);
    return st;
}

int kco_count_pair_sampled(const kco_graph *g, int k, uint64_t t, uint64_t seed, int threads, uint64_t *raw) {
    if (!g || !raw || k < 3) return KCO_EINVAL;
    uint64_t *cc = (uint64_t *)malloc(sizeof(uint64_t) * (g->n ? g->n : 1));
    if (!cc) return KCO_ENOMEM;
    int status = KCO_OK;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
    #pragma omp parallel for schedule(dynamic, 16) num_threads(threads)
#endif
    for (int64_t x = 0; x < (int64_t)g->n; ++x) {
        int st = kco_count_pair_sampled_root(g, (uint32_t)x, k, t, seed, &cc[x]);
        if (st) {
            #pragma omp critical
            status = st;
        }
    }
    (void)threads;
    uint64_t total = 0;
    for (uint32_t x = 0; status == KCO_OK && x < g->n; ++x)
        if (__builtin_add_overflow(total, cc[x], &total)) status = KCO_EOVERFLOW;
    free(cc);
    if (status == KCO_OK) *raw = total;
    return status;
}

/* ------------------------------------------------------------------------- */
/* Per-root work.  Running cnt(Gamma+(u), k-1) performs one intersection for
 * every l-clique of G+(u) with 1 <= l <= k-2 (the clique's last node v is the
 * node whose neighbourhood is intersected).  `inter` counts them.  `words`
 * weights each one by the 64-bit words that a bitmap row of G+(u) spans above
 * v's local position i (bits i+1 .. d-1):  floor((d-1)/64) - floor((i+1)/64) + 1
 * when i + 1 <= d - 1, else 0. */
static int work_rec(const kco_graph *g, const uint32_t *L, const uint32_t *Lidx, uint64_t np, int l, uint64_t d,
                    uint32_t *buf, uint32_t *ibuf, uint64_t *inter, uint64_t *words) {
    if (l < 2) return KCO_OK;
    for (uint64_t i = 0; i < np; ++i) {
        uint64_t li = Lidx[i];
        uint64_t wc = (li + 1 <= d - 1) ? ((d - 1) / 64 - (li + 1) / 64 + 1) : 0;
        if (__builtin_add_overflow(*inter, 1, inter)) return KCO_EOVERFLOW;
        if (__builtin_add_overflow(*words, wc, words)) return KCO_EOVERFLOW;
        /* children: L n Gamma+(L[i]) with their local indices */
        uint64_t nq = 0;
        const uint32_t *N = g->hn + g->hp[L[i]];
        uint64_t nn = g->hp[L[i] + 1] - g->hp[L[i]], a = 0, b = 0;
        while (a < np && b < nn) {
            uint64_t ka = key_of(g, L[a]), kb = key_of(g, N[b]);
            if (ka < kb) ++a;
            else if (kb < ka) ++b;
            else { buf[nq] = L[a]; ibuf[nq] = Lidx[a]; ++nq; ++a; ++b; }
        }
        int st = work_rec(g, buf, ibuf, nq, l - 1, d, buf + np, ibuf + np, inter, words);
        if (st) return st;
    }
    return KCO_OK;
}

int kco_work_root(const kco_graph *g, uint32_t u, int k, uint64_t *inter, uint64_t *words) {
    if (!g || u >= g->n || k < 1 || !inter || !words) return KCO_EINVAL;
    uint64_t d = g->hp[u + 1] - g->hp[u];
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * ((uint64_t)k * d + 1));
    uint32_t *ibuf = (uint32_t *)malloc(sizeof(uint32_t) * ((uint64_t)k * d + 1));
    uint32_t *idx = (uint32_t *)malloc(sizeof(uint32_t) * (d + 1));
    if (!buf || !ibuf || !idx) { free(buf); free(ibuf); free(idx); return KCO_ENOMEM; }
    for (uint64_t i = 0; i < d; ++i) idx[i] = (uint32_t)i;
    *inter = 0;
    *words = 0;
    int st = work_rec(g, g->hn + g->hp[u], idx, d, k - 1, d, buf, ibuf, inter, words);
    free(buf); free(ibuf); free(idx);
    return st;
}

int kco_work_per_root(const kco_graph *g, int k, int threads, uint64_t *inter, uint64_t *words) {
    if (!g || !inter || !words || k < 1) return KCO_EINVAL;
    int status = KCO_OK;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
    #pragma omp parallel for schedule(dynamic, 16) num_threads(threads)
#endif
    for (int64_t x = 0; x < (int64_t)g->n; ++x) {
        int st = kco_work_root(g, (uint32_t)x, k, &inter[x], &words[x]);
        if (st) {
            #pragma omp critical
            status = st;
        }
    }
    (void)threads;
    return status;
}

/* ------------------------------------------------------------------------- */
/* Per-node clique-membership counts.
 *
 * Section 3 notes that the round-3 reducer of root u can also report, for each
 * node v, how many of the cliques it finds contain v, and that summing these
 * reports over all sub-problems G+(u) gives the number of k-cliques that contain
 * v.  kco_count_per_node follows that route: every (k-1)-clique of G+(u) is listed
 * explicitly (the same intersection recursion as cnt, with the chosen nodes kept
 * on a path) and adds one to u and to each of its own nodes.
 *
 * kco_count_node is the plain definition instead: the k-cliques that contain v
 * are the (k-1)-cliques inside the neighbourhood Gamma(v); Gamma(v) is sorted by
 * the order and counted with cnt (each clique once, by its smallest node). */
static int add_checked(uint64_t *c, uint64_t x) {
    uint64_t old;
    #pragma omp atomic capture
    { old = *c; *c += x; }
    return old + x < old ? KCO_EOVERFLOW : KCO_OK;
}

/* List the l-cliques inside P (sorted by the order); each adds one to the nodes on
 * the path (depth entries) and to its own. */
static int list_attr(const kco_graph *g, const uint32_t *P, uint64_t np, int l, uint32_t *buf, uint32_t *path,
                     int depth, uint64_t *counts) {
    if (l <= 0) {
        for (int t = 0; t < depth; ++t) {
            int st = add_checked(&counts[path[t]], 1);
            if (st) return st;
        }
        return KCO_OK;
    }
    for (uint64_t i = 0; i < np; ++i) {
        path[depth] = P[i];
        uint64_t nq = intersect(g, P, np, P[i], buf);
        int st = list_attr(g, buf, nq, l - 1, buf + np, path, depth + 1, counts);
        if (st) return st;
    }
    return KCO_OK;
}

int kco_count_per_node(const kco_graph *g, int k, int threads, uint64_t *counts) {
    if (!g || !counts || k < 1) return KCO_EINVAL;
    memset(counts, 0, sizeof(uint64_t) * g->n);
    int status = KCO_OK;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
    #pragma omp parallel for schedule(dynamic, 16) num_threads(threads)
#endif
    for (int64_t x = 0; x < (int64_t)g->n; ++x) {
        uint32_t u = (uint32_t)x;
        uint64_t d = g->hp[u + 1] - g->hp[u];
        uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * ((uint64_t)k * d + 1));
        uint32_t *path = (uint32_t *)malloc(sizeof(uint32_t) * ((uint64_t)k + 1));
        int st = (!buf || !path) ? KCO_ENOMEM : KCO_OK;
        if (st == KCO_OK) {
            path[0] = u;  /* the root belongs to every clique of its sub-problem */
            st = list_attr(g, g->hn + g->hp[u], d, k - 1, buf, path, 1, counts);
        }
        free(buf);
        free(path);
        if (st) {
            #pragma omp critical
            status = st;
        }
    }
    (void)threads;
    return status;
}

static const kco_graph *sort_graph;  /* qsort has no context argument */
static int cmp_by_order(const void *a, const void *b) {
    uint64_t x = key_of(sort_graph, *(const uint32_t *)a), y = key_of(sort_graph, *(const uint32_t *)b);
    return (x > y) - (x < y);
}

int kco_count_node(const kco_graph *g, uint32_t v, int k, uint64_t *out) {
    if (!g || !out || v >= g->n || k < 1) return KCO_EINVAL;
    uint64_t dv = g->deg[v];
    uint32_t *nb = (uint32_t *)malloc(sizeof(uint32_t) * (dv + 1));
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * ((uint64_t)k * dv + 1));
    if (!nb || !buf) { free(nb); free(buf); return KCO_ENOMEM; }
    uint64_t c = 0;
    for (uint64_t i = 0; i < g->m; ++i) {
        if (g->eu[i] == v) nb[c++] = g->ev[i];
        else if (g->ev[i] == v) nb[c++] = g->eu[i];
    }
    int st = KCO_OK;
    #pragma omp critical(kco_sort)
    {
        sort_graph = g;
        qsort(nb, c, sizeof(uint32_t), cmp_by_order);
    }
    st = cnt(g, nb, c, k - 1, buf, out);
    free(nb);
    free(buf);
    return st;
}
