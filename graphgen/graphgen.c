/*
 * Seeded synthetic graph generators.
 *
 * These produce raw undirected edge lists (src[i], dst[i]) that may contain
 * self-loops and repeated pairs; canonicalisation is the job of the consumer.
 * They stand in for the social and web graphs the paper measures (its Section 4,
 * Table 1), which are not available here.  The module holds no clique-counting
 * arithmetic: no degrees, no orientation, no counting.  Both the CPU oracle and
 * the GPU library consume its output, so it shares code with neither.
 *
 * Randomness: a counter-based stream built on the SplitMix64 finaliser
 * (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014):  r(seed, s, i) = mix64(seed ^ mix64((s << 48) ^ i)),
 * u01(r) = (r >> 11) * 2^-53.  Every draw is addressed by (stream, index), so
 * the output does not depend on the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t gg_mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t gg_rand(uint64_t seed, uint64_t stream, uint64_t i) {
    return gg_mix64(seed ^ gg_mix64((stream << 48) ^ i));
}

static inline double gg_u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

/* uniform integer in [0, n) by multiply-high of the top 32 bits (n < 2^32) */
static inline uint32_t gg_below(uint64_t r, uint32_t n) {
    return (uint32_t)(((r >> 32) * (uint64_t)n) >> 32);
}

uint64_t gg_mix64_export(uint64_t z) { return gg_mix64(z); }
uint64_t gg_rand_export(uint64_t seed, uint64_t stream, uint64_t i) { return gg_rand(seed, stream, i); }

/* ------------------------------------------------------------------------- */
/* Erdos-Renyi G(n, p): the lexicographic pair t = (u, v), u < v, is kept iff
 * u01(r(seed, 0, t)) < p.  With out == NULL only the edge count is returned. */
uint64_t gg_er(uint32_t n, double p, uint64_t seed, uint32_t *src, uint32_t *dst) {
    uint64_t t = 0, e = 0;
    for (uint32_t u = 0; u < n; ++u)
        for (uint32_t v = u + 1; v < n; ++v, ++t)
            if (gg_u01(gg_rand(seed, 0, t)) < p) {
                if (src) { src[e] = u; dst[e] = v; }
                ++e;
            }
    return e;
}

/* ------------------------------------------------------------------------- */
/* Truncated power law on [wmin, wmax] with density proportional to w^-gamma. */
static double tp_mean(double wmin, double wmax, double g) {
    /* mean = int w^{1-g} / int w^{-g} over [wmin, wmax] */
    double num, den;
    if (fabs(g - 2.0) < 1e-12) num = log(wmax / wmin);
    else num = (pow(wmax, 2.0 - g) - pow(wmin, 2.0 - g)) / (2.0 - g);
    if (fabs(g - 1.0) < 1e-12) den = log(wmax / wmin);
    else den = (pow(wmax, 1.0 - g) - pow(wmin, 1.0 - g)) / (1.0 - g);
    return num / den;
}

/* Solve wmin so that the truncated power law has the requested mean (bisection;
 * the mean is increasing in wmin).  Returns <= 0 when no solution exists. */
double gg_solve_wmin(double mean, double wmax, double g) {
    double lo = 1e-9, hi = mean;
    if (!(mean < wmax)) return -1.0;
    if (tp_mean(lo, wmax, g) > mean) return -1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (tp_mean(mid, wmax, g) < mean) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static inline double tp_sample(double u, double wmin, double wmax, double g) {
    /* inverse CDF */
    if (fabs(g - 1.0) < 1e-12) return wmin * pow(wmax / wmin, u);
    double a = pow(wmin, 1.0 - g), b = pow(wmax, 1.0 - g);
    return pow(a - u * (a - b), 1.0 / (1.0 - g));
}

/* Chung-Lu weights: w_i = inverse-CDF(u01(r(seed, 1, i))).  Returns the sum. */
double gg_weights(uint32_t n, double gamma, double mean, double wmax, uint64_t seed, double *w) {
    double wmin = gg_solve_wmin(mean, wmax, gamma);
    if (wmin <= 0) return -1.0;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i)
        w[i] = tp_sample(gg_u01(gg_rand(seed, 1, (uint64_t)i)), wmin, wmax, gamma);
    double s = 0.0;
    for (uint32_t i = 0; i < n; ++i) s += w[i]; /* sequential: fixed summation order */
    return s;
}

/* Vose alias table (sequential, deterministic). */
static void alias_build(uint32_t n, const double *w, double wsum, double *prob, uint32_t *alias) {
    double *scaled = (double *)malloc(sizeof(double) * n);
    uint32_t *small = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *large = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t ns = 0, nl = 0;
    for (uint32_t i = 0; i < n; ++i) {
        scaled[i] = w[i] * (double)n / wsum;
        if (scaled[i] < 1.0) small[ns++] = i; else large[nl++] = i;
    }
    while (ns && nl) {
        uint32_t s = small[--ns], l = large[--nl];
        prob[s] = scaled[s];
        alias[s] = l;
        scaled[l] = (scaled[l] + scaled[s]) - 1.0;
        if (scaled[l] < 1.0) small[ns++] = l; else large[nl++] = l;
    }
    while (nl) { uint32_t l = large[--nl]; prob[l] = 1.0; alias[l] = l; }
    while (ns) { uint32_t s = small[--ns]; prob[s] = 1.0; alias[s] = s; }
    free(scaled); free(small); free(large);
}

/* Number of endpoint pairs the Chung-Lu draw emits for these parameters
 * (round(sum w / 2)), or -1 if the parameters admit no weight law. */
int64_t gg_chung_lu_edges(uint32_t n, double gamma, double mean, double wmax, uint64_t seed) {
    double *w = (double *)malloc(sizeof(double) * (n ? n : 1));
    double s = gg_weights(n, gamma, mean, wmax, seed, w);
    free(w);
    if (s < 0) return -1;
    return (int64_t)llround(s / 2.0);
}

/* Fast Chung-Lu: M = round(sum w / 2) endpoint pairs, each endpoint drawn
 * proportionally to w through an alias table: column from r(seed, 2, 2e+j),
 * coin from r(seed, 3, 2e+j), j in {0,1}.  Raw output (self-loops and repeats
 * kept).  Caller sizes src/dst with gg_chung_lu_edges. */
int64_t gg_chung_lu(uint32_t n, double gamma, double mean, double wmax, uint64_t seed,
                    uint32_t *src, uint32_t *dst) {
    double *w = (double *)malloc(sizeof(double) * (n ? n : 1));
    double s = gg_weights(n, gamma, mean, wmax, seed, w);
    if (s < 0) { free(w); return -1; }
    int64_t M = (int64_t)llround(s / 2.0);
    double *prob = (double *)malloc(sizeof(double) * n);
    uint32_t *alias = (uint32_t *)malloc(sizeof(uint32_t) * n);
    alias_build(n, w, s, prob, alias);
    free(w);
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < M; ++e) {
        uint32_t ends[2];
        for (int j = 0; j < 2; ++j) {
            uint64_t idx = 2 * (uint64_t)e + (uint64_t)j;
            uint32_t col = gg_below(gg_rand(seed, 2, idx), n);
            double coin = gg_u01(gg_rand(seed, 3, idx));
            ends[j] = (coin < prob[col]) ? col : alias[col];
        }
        src[e] = ends[0];
        dst[e] = ends[1];
    }
    free(prob); free(alias);
    return M;
}

/* ------------------------------------------------------------------------- */
/* Planted cliques: `count` cliques of `size` distinct nodes drawn uniformly from
 * [0, n) (member t of clique c from r(seed, 4, c * 2^20 + attempt)); emits the
 * size*(size-1)/2 pairs of each clique.  Cliques may overlap. */
int64_t gg_planted(uint32_t n, uint32_t count, uint32_t size, uint64_t seed,
                   uint32_t *src, uint32_t *dst) {
    if (size > n || size > 4096) return -1;
    uint32_t *mem = (uint32_t *)malloc(sizeof(uint32_t) * (size ? size : 1));
    int64_t e = 0;
    for (uint32_t c = 0; c < count; ++c) {
        uint32_t have = 0;
        uint64_t attempt = 0;
        while (have < size) {
            uint32_t x = gg_below(gg_rand(seed, 4, ((uint64_t)c << 20) + attempt), n);
            ++attempt;
            int dup = 0;
            for (uint32_t t = 0; t < have; ++t) if (mem[t] == x) { dup = 1; break; }
            if (!dup) mem[have++] = x;
        }
        for (uint32_t i = 0; i < size; ++i)
            for (uint32_t j = i + 1; j < size; ++j) {
                if (src) { src[e] = mem[i]; dst[e] = mem[j]; }
                ++e;
            }
    }
    free(mem);
    return e;
}

/* ------------------------------------------------------------------------- */
/* R-MAT (Chakrabarti, Zhan & Faloutsos 2004): ef * 2^scale draws; level L of
 * draw e picks a quadrant from u01(r(seed, 5, e * scale + L)) with
 * probabilities (a, b, c, 1-a-b-c).  If permute, labels pass through a seeded
 * Fisher-Yates permutation (swap index from r(seed, 6, i)).  Raw output. */
int64_t gg_rmat(uint32_t scale, uint32_t ef, double a, double b, double c, uint64_t seed,
                int permute, uint32_t *src, uint32_t *dst) {
    if (scale == 0 || scale > 31) return -1;
    uint32_t n = 1u << scale;
    int64_t M = (int64_t)ef << scale;
    uint32_t *perm = NULL;
    if (permute) {
        perm = (uint32_t *)malloc(sizeof(uint32_t) * n);
        for (uint32_t i = 0; i < n; ++i) perm[i] = i;
        for (uint32_t i = n - 1; i > 0; --i) {
            uint32_t j = gg_below(gg_rand(seed, 6, i), i + 1);
            uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
    }
    double ab = a + b, abc = a + b + c;
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < M; ++e) {
        uint32_t u = 0, v = 0;
        for (uint32_t L = 0; L < scale; ++L) {
            double r = gg_u01(gg_rand(seed, 5, (uint64_t)e * scale + L));
            uint32_t bu, bv;
            if (r < a) { bu = 0; bv = 0; }
            else if (r < ab) { bu = 0; bv = 1; }
            else if (r < abc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        if (perm) { u = perm[u]; v = perm[v]; }
        src[e] = u;
        dst[e] = v;
    }
    free(perm);
    return M;
}

/* ------------------------------------------------------------------------- */
/* Node count of graph i of a log-uniform batch: floor(exp(ln nlo + u ln(nhi/nlo))),
 * u = u01(r(seed, 7, i)). */
uint32_t gg_batch_n(uint64_t seed, uint32_t i, double nlo, double nhi) {
    double u = gg_u01(gg_rand(seed, 7, i));
    return (uint32_t)floor(exp(log(nlo) + u * log(nhi / nlo)));
}
