// Learned scheduler: an 8 -> 32 -> 32 -> 1 ReLU MLP (fp32) that predicts
// log(1 + per-root work) from cheap per-root features, trained on GPU on the
// work the exact counter measures (kc_count_per_root).
//
// The paper shows the reduce-3 instances are heavily skewed and that the slow
// ones should be spread over more workers (Sections 5 and 7).  The prediction
// orders the queue heaviest first and moves small but dense roots to the
// workgroup tier; the degree order is the fallback and the yardstick.
//
// Features of root u (rank space), for clique size k:
//   0 log1p d+(u)            1 log1p sum_{x in Gamma+(u)} d+(x)  (wedges)
//   2 log1p max d+(x)        3 log1p d(u)
//   4 log1p e+(u)            5 e+(u) / C(d+(u), 2)   (e+ = edges of G+(u))
//   6 k / 10                 7 log C(d+, k-1) + C(k-1, 2) log(density)
// e+(u) is the per-root count at k = 3 (one staging pass, cached per graph).
// Weight file: "KCMLP001", u32 params, 8 means, 8 stds, label mean, label std,
// then the parameters W1[32][8] b1[32] W2[32][32] b2[32] w3[32] b3.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "kc_internal.h"

namespace {

constexpr int NF = KC_MLP_IN, H = KC_MLP_H, NP = KC_MLP_PARAMS;
constexpr int OFF_W1 = 0, OFF_B1 = NF * H, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H,
              OFF_B3 = OFF_W3 + H;
constexpr int NORM = 2 * NF + 2;  // feature means, stds, label mean, std
constexpr int T = 256;
inline unsigned grid_for(size_t n) { return (unsigned)((n + T - 1) / T); }

// log of the expected (k-1)-cliques of G+(u) for an Erdos-Renyi graph of its size
// and edge density: log C(d, k-1) + C(k-1, 2) log(density), clamped to [-10, 60]
__device__ __forceinline__ double log_cliques(uint32_t d, double dens, int k) {
    double lc = -10.0;
    if (d >= (uint32_t)(k - 1) && dens > 0) {
        const double r = k - 1;
        lc = lgamma((double)d + 1.0) - lgamma(r + 1.0) - lgamma((double)d - r + 1.0) + 0.5 * r * (r - 1.0) * log(dens);
        lc = lc < -10.0 ? -10.0 : (lc > 60.0 ? 60.0 : lc);
    }
    return lc;
}

// The eight features of root u (rank space) for clique size k; ep = edges of G+(u).
__device__ __forceinline__ void root_features(uint32_t u, const uint64_t *optr, const uint32_t *ocol, uint32_t deg_u,
                                              double ep, int k, float *f) {
    const uint64_t b = optr[u], e = optr[u + 1];
    const uint32_t d = (uint32_t)(e - b);
    double wedges = 0.0;
    uint32_t mx = 0;
    for (uint64_t p = b; p < e; ++p) {
        const uint32_t x = ocol[p];
        const uint32_t dx = (uint32_t)(optr[x + 1] - optr[x]);
        wedges += dx;
        mx = dx > mx ? dx : mx;
    }
    const double pairs = d >= 2 ? 0.5 * (double)d * (double)(d - 1) : 0.0;
    const double dens = pairs > 0 ? ep / pairs : 0.0;
    const double lc = log_cliques(d, dens, k);
    f[0] = (float)log1p((double)d);
    f[1] = (float)log1p(wedges);
    f[2] = (float)log1p((double)mx);
    f[3] = (float)log1p((double)deg_u);
    f[4] = (float)log1p(ep);
    f[5] = (float)dens;
    f[6] = (float)k / 10.0f;
    f[7] = (float)lc;
}

// every root, edges of G+(u) from the per-root k = 3 counts (by original id)
__global__ void k_features(const uint64_t *optr, const uint32_t *ocol, const uint32_t *rank2id, const uint32_t *deg,
                           const uint64_t *tri_by_id, uint32_t n, int k, float *feat) {
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const uint32_t id = rank2id[u];
    root_features((uint32_t)u, optr, ocol, deg[id], (double)tri_by_id[id], k, feat + u * NF);
}

// roots list[lo, hi) (ranks), edges of G+(u) from the staged cache: the bitmap's edge
// count for roots above the one-wave limit, the popcounts of the staged rows below it
__global__ void k_features_list(const uint32_t *list, uint32_t lo, uint32_t hi, const uint64_t *optr,
                                const uint32_t *ocol, const uint32_t *rank2id, const uint32_t *deg,
                                const uint64_t *lrows, const uint32_t *wedges, uint32_t stage_wd, float *feat) {
    const size_t i = lo + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= hi) return;
    const uint32_t u = list[i];
    const uint64_t b = optr[u];
    const uint32_t d = (uint32_t)(optr[u + 1] - b);
    double ep = 0.0;
    if (d > stage_wd) {
        ep = (double)wedges[u];
    } else if (d >= 2) {  // roots of out-degree 0 and 1 are never staged
        uint64_t c = 0;
        for (uint32_t j = 0; j < d; ++j) c += (uint64_t)__popcll(lrows[b + j]);
        ep = (double)c;
    }
    root_features(u, optr, ocol, deg[rank2id[u]], ep, 4, feat + (size_t)u * NF);
}

__device__ __forceinline__ float mlp_forward(const float *P, const float *x, float *h1, float *z1, float *h2,
                                             float *z2) {
#pragma unroll 4
    for (int j = 0; j < H; ++j) {
        float s = P[OFF_B1 + j];
#pragma unroll
        for (int i = 0; i < NF; ++i) s += P[OFF_W1 + j * NF + i] * x[i];
        z1[j] = s;
        h1[j] = s > 0.f ? s : 0.f;
    }
    for (int j = 0; j < H; ++j) {
        float s = P[OFF_B2 + j];
#pragma unroll 8
        for (int i = 0; i < H; ++i) s += P[OFF_W2 + j * H + i] * h1[i];
        z2[j] = s;
        h2[j] = s > 0.f ? s : 0.f;
    }
    float y = P[OFF_B3];
#pragma unroll 8
    for (int j = 0; j < H; ++j) y += P[OFF_W3 + j] * h2[j];
    return y;
}

// inference: pred[u] = predicted log1p(work) of root u (raw features, normalised here)
// Inference from features cached without k: the two k-dependent ones (k / 10 and
// the log expected cliques) are computed here.
__global__ void __launch_bounds__(T) k_mlp_infer_k(const float *feat, uint32_t n, int k, const uint64_t *optr,
                                                   const float *params, float *pred) {
    __shared__ float P[NP + NORM];
    for (int i = threadIdx.x; i < NP + NORM; i += blockDim.x) P[i] = params[i];
    __syncthreads();
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const float *norm = P + NP;
    float f[NF], x[NF], h1[H], z1[H], h2[H], z2[H];
#pragma unroll
    for (int i = 0; i < NF; ++i) f[i] = feat[u * NF + i];
    f[6] = (float)k / 10.0f;
    f[7] = (float)log_cliques((uint32_t)(optr[u + 1] - optr[u]), (double)f[5], k);
#pragma unroll
    for (int i = 0; i < NF; ++i) x[i] = (f[i] - norm[i]) / norm[NF + i];
    const float y = mlp_forward(P, x, h1, z1, h2, z2);
    pred[u] = y * norm[2 * NF + 1] + norm[2 * NF];
}

// Learned queue of one clique size: inference for the candidate roots dq[0, C) and
// their sort keys, tier (0 scratch, 1 workgroup, 2 one-wave) | 24-bit complement of
// the predicted log-work | rank.  One-wave roots whose predicted log-work reaches
// `promote` move to the workgroup tier.  stats: [0..2] roots per tier, [4..6] the
// largest out-degree per tier.
__global__ void __launch_bounds__(T) k_learned_cand(const uint32_t *dq, uint32_t C, const float *feat, int k,
                                                    const uint64_t *optr, const float *params, uint32_t wd,
                                                    uint32_t dcap, float promote, uint64_t *keys, uint32_t *stats) {
    __shared__ float P[NP + NORM];
    __shared__ uint32_t s_c[3], s_m[3];
    for (int i = threadIdx.x; i < NP + NORM; i += blockDim.x) P[i] = params[i];
    if (threadIdx.x < 3) s_c[threadIdx.x] = s_m[threadIdx.x] = 0;
    __syncthreads();
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t tier = 3, d = 0;
    if (i < C) {
        const uint32_t u = dq[i];
        d = (uint32_t)(optr[u + 1] - optr[u]);
        tier = d > dcap ? 0u : (d > wd ? 1u : 2u);
        const float *norm = P + NP;
        float f[NF], x[NF], h1[H], z1[H], h2[H], z2[H];
#pragma unroll
        for (int j = 0; j < NF; ++j) f[j] = feat[(size_t)u * NF + j];
        f[6] = (float)k / 10.0f;
        f[7] = (float)log_cliques(d, (double)f[5], k);
#pragma unroll
        for (int j = 0; j < NF; ++j) x[j] = (f[j] - norm[j]) / norm[NF + j];
        const float w = mlp_forward(P, x, h1, z1, h2, z2) * norm[2 * NF + 1] + norm[2 * NF];
        if (tier == 2 && w >= promote) tier = 1;
        keys[i] = ((uint64_t)tier << 62) | ((uint64_t)kc_learned_prio(w) << 32) | (uint64_t)u;
    }
#pragma unroll
    for (uint32_t t = 0; t < 3; ++t) {
        const bool in = tier == t;
        const uint32_t c = (uint32_t)__popcll(__ballot(in));
        const uint32_t m = kc_wave_max_u32(in ? d : 0u);
        if ((threadIdx.x & 63) == 0 && c) {
            atomicAdd(&s_c[t], c);
            atomicMax(&s_m[t], m);
        }
    }
    __syncthreads();
    if (threadIdx.x < 3 && s_c[threadIdx.x]) {
        atomicAdd(&stats[threadIdx.x], s_c[threadIdx.x]);
        atomicMax(&stats[4 + threadIdx.x], s_m[threadIdx.x]);
    }
}

// One mini-batch gradient: 64 samples per block (one wave), per-block sums of the
// parameter gradients of 0.5 * mean (y - t)^2, added to grad with atomics.  Sample s
// of the batch is row order[start + s] of X (row start + s without an order);
// loss += sum of 0.5 (y - t)^2 over the batch.
constexpr int GB = 64;
__global__ void __launch_bounds__(GB) k_mlp_grad(const float *X, const float *Tg, const uint32_t *order, size_t start,
                                                 size_t count, const float *params, float *grad, float *loss) {
    __shared__ float P[NP];
    __shared__ float sx[GB][NF], sh1[GB][H], sd1[GB][H], sh2[GB][H], sd2[GB][H], sdy[GB];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) P[i] = params[i];
    __syncthreads();
    const size_t s = (size_t)blockIdx.x * GB + threadIdx.x;
    const int t = threadIdx.x;
    float x[NF], h1[H], z1[H], h2[H], z2[H];
    float dy = 0.f;
    if (s < count) {
        const size_t idx = order ? (size_t)order[start + s] : start + s;
#pragma unroll
        for (int i = 0; i < NF; ++i) x[i] = X[idx * NF + i];
        const float y = mlp_forward(P, x, h1, z1, h2, z2);
        const float err = y - Tg[idx];
        dy = err / (float)count;
        atomicAdd(loss, 0.5f * err * err);
    } else {
#pragma unroll
        for (int i = 0; i < NF; ++i) x[i] = 0.f;
        for (int j = 0; j < H; ++j) h1[j] = z1[j] = h2[j] = z2[j] = 0.f;
    }
    // backward for this sample
    float d2[H], d1[H];
    for (int j = 0; j < H; ++j) d2[j] = z2[j] > 0.f ? dy * P[OFF_W3 + j] : 0.f;
    for (int i = 0; i < H; ++i) {
        float sacc = 0.f;
        for (int j = 0; j < H; ++j) sacc += P[OFF_W2 + j * H + i] * d2[j];
        d1[i] = z1[i] > 0.f ? sacc : 0.f;
    }
    for (int i = 0; i < NF; ++i) sx[t][i] = x[i];
    for (int j = 0; j < H; ++j) {
        sh1[t][j] = h1[j];
        sd1[t][j] = d1[j];
        sh2[t][j] = h2[j];
        sd2[t][j] = d2[j];
    }
    sdy[t] = dy;
    __syncthreads();
    // block sums of outer products, one parameter per thread at a time
    for (int pidx = t; pidx < NP; pidx += GB) {
        float g = 0.f;
        if (pidx < OFF_B1) {
            const int j = pidx / NF, i = pidx % NF;
            for (int q = 0; q < GB; ++q) g += sd1[q][j] * sx[q][i];
        } else if (pidx < OFF_W2) {
            const int j = pidx - OFF_B1;
            for (int q = 0; q < GB; ++q) g += sd1[q][j];
        } else if (pidx < OFF_B2) {
            const int j = (pidx - OFF_W2) / H, i = (pidx - OFF_W2) % H;
            for (int q = 0; q < GB; ++q) g += sd2[q][j] * sh1[q][i];
        } else if (pidx < OFF_W3) {
            const int j = pidx - OFF_B2;
            for (int q = 0; q < GB; ++q) g += sd2[q][j];
        } else if (pidx < OFF_B3) {
            const int j = pidx - OFF_W3;
            for (int q = 0; q < GB; ++q) g += sdy[q] * sh2[q][j];
        } else {
            for (int q = 0; q < GB; ++q) g += sdy[q];
        }
        atomicAdd(&grad[pidx], g);
    }
}

__global__ void k_adam(float *params, float *grad, float *m, float *v, int step, float lr) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    for (int i = threadIdx.x; i < NP; i += blockDim.x) {
        const float g = grad[i];
        m[i] = b1 * m[i] + (1.f - b1) * g;
        v[i] = b2 * v[i] + (1.f - b2) * g * g;
        params[i] -= lr * (m[i] / c1) / (sqrtf(v[i] / c2) + eps);
        grad[i] = 0.f;
    }
}

// gather samples of active roots: X row = features (raw), T = log1p(work)
__global__ void k_gather(const float *feat, const uint64_t *optr, const uint32_t *rank2id, const uint64_t *work_by_id,
                         uint32_t n, int k, const uint32_t *pos, float *X, float *Tv) {
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const uint32_t d = (uint32_t)(optr[u + 1] - optr[u]);
    if (d < (uint32_t)(k - 1)) return;
    const uint32_t o = pos[u];
    for (int i = 0; i < NF; ++i) X[(size_t)o * NF + i] = feat[u * NF + i];
    Tv[o] = (float)log1p((double)work_by_id[rank2id[u]]);
}

__global__ void k_active_flags(const uint64_t *optr, uint32_t n, int k, uint32_t *flag) {
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) flag[u] = (optr[u + 1] - optr[u]) >= (uint64_t)(k - 1) ? 1u : 0u;
}

// per-root edges of G+(u) (the k = 3 per-root count), cached on the handle
kc_status ensure_tri(const kc_graph *g) {
    kc_graph *gm = const_cast<kc_graph *>(g);
    if (gm->tri) return KC_OK;
    uint64_t *t = nullptr;
    KC_TRY(kc_dev_alloc((void **)&t, (size_t)g->n * 8, g->stream));
    kc_count_args a;
    a.k = 3;
    a.per_root = t;
    a.policy = KC_SCHED_DEGREE;
    uint64_t total = 0;
    int ovf = 0;
    kc_status st = kc_count_impl(g, a, &total, &ovf);
    if (st != KC_OK) {
        kc_cache_free(t, g->stream);
        return st;
    }
    gm->tri = t;
    return KC_OK;
}

kc_status features(const kc_graph *g, int k, float *feat, hipStream_t s) {
    KC_TRY(ensure_tri(g));
    hipLaunchKernelGGL(k_features, dim3(grid_for(g->n)), dim3(T), 0, s, (const uint64_t *)g->optr,
                       (const uint32_t *)g->ocol, (const uint32_t *)g->rank2id, (const uint32_t *)g->deg,
                       (const uint64_t *)g->tri, g->n, k, feat);
    KC_HIP(hipGetLastError());
    return KC_OK;
}

}  // namespace

// Features of the first `upto` roots of the degree queue, kept on the handle
// (rank order): from the staged cache when it is kept, else from per-root k = 3
// counts.  Later calls compute only the roots past the cached prefix.
static kc_status features_prefix(const kc_graph *g, uint32_t upto, hipStream_t s) {
    kc_graph *gm = const_cast<kc_graph *>(g);
    if (gm->feat_dqwd != g->dq_wd) gm->feat_upto = 0;
    if (upto <= gm->feat_upto) return KC_OK;
    if (!gm->feat) KC_TRY(kc_dev_alloc((void **)&gm->feat, (size_t)g->n * NF * 4, s));
    const bool cached = g->staged == 1 && g->stage_wd == g->dq_wd && g->wedges && g->lrows;
    if (cached) {
        const uint32_t lo = gm->feat_upto;
        hipLaunchKernelGGL(k_features_list, dim3(grid_for(upto - lo)), dim3(T), 0, s, (const uint32_t *)g->dq, lo,
                           upto, (const uint64_t *)g->optr, (const uint32_t *)g->ocol, (const uint32_t *)g->rank2id,
                           (const uint32_t *)g->deg, (const uint64_t *)g->lrows, (const uint32_t *)g->wedges,
                           (uint32_t)g->stage_wd, gm->feat);
        KC_HIP(hipGetLastError());
        gm->feat_upto = upto;
    } else {
        KC_TRY(features(g, 4, gm->feat, s));  // every root
        gm->feat_upto = 0xFFFFFFFFu;
    }
    gm->feat_dqwd = g->dq_wd;
    return KC_OK;
}

kc_status kc_learned_keys(const kc_graph *g, int k, uint32_t C, uint32_t wd, uint32_t dcap, float promote,
                          uint64_t *keys, uint32_t *stats, hipStream_t s) {
    if (!g->mlp_loaded) return kc_fail(KC_ESTATE, "no scheduler weights loaded");
    if (C == 0) return KC_OK;
    KC_TRY(features_prefix(g, C, s));
    hipLaunchKernelGGL(k_learned_cand, dim3(grid_for(C)), dim3(T), 0, s, (const uint32_t *)g->dq, C,
                       (const float *)g->feat, k, (const uint64_t *)g->optr, (const float *)g->mlp, wd, dcap, promote,
                       keys, stats);
    KC_HIP(hipGetLastError());
    return KC_OK;
}

namespace {
// predictions of every root at clique size k, written by original id
__global__ void k_predict_by_id(const float *feat, uint32_t n, int k, const uint64_t *optr, const uint32_t *rank2id,
                                const float *params, float *pred, float *feat_out) {
    __shared__ float P[NP + NORM];
    for (int i = threadIdx.x; i < NP + NORM; i += blockDim.x) P[i] = params[i];
    __syncthreads();
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const uint32_t d = (uint32_t)(optr[u + 1] - optr[u]);
    const uint32_t id = rank2id[u];
    const float *norm = P + NP;
    float f[NF], x[NF], h1[H], z1[H], h2[H], z2[H];
#pragma unroll
    for (int i = 0; i < NF; ++i) f[i] = feat[u * NF + i];
    f[6] = (float)k / 10.0f;
    f[7] = (float)log_cliques(d, (double)f[5], k);
    if (feat_out) {
#pragma unroll
        for (int i = 0; i < NF; ++i) feat_out[(size_t)id * NF + i] = f[i];
    }
    if (d < (uint32_t)(k - 1)) {
        pred[id] = 0.f;
        return;
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) x[i] = (f[i] - norm[i]) / norm[NF + i];
    pred[id] = mlp_forward(P, x, h1, z1, h2, z2) * norm[2 * NF + 1] + norm[2 * NF];
}
}  // namespace

extern "C" kc_status kc_predict_work(const kc_graph *g, int32_t k, float *dev_pred, float *dev_feat) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (!dev_pred) return kc_fail(KC_EINVAL, "dev_pred is NULL");
    if (k < 3 || k > KC_KMAX) return kc_fail(KC_EINVAL, "k=%d outside [3, %d]", k, KC_KMAX);
    if (!g->oriented) return kc_fail(KC_ESTATE, "kc_orient has not been called");
    if (!g->mlp_loaded) return kc_fail(KC_ESTATE, "no scheduler weights loaded");
    hipStream_t s = g->stream;
    kc_tmp feat;
    KC_TRY(kc_tmp_alloc(feat, (size_t)g->n * NF * 4, s));
    KC_TRY(features(g, 4, feat.as<float>(), s));
    hipLaunchKernelGGL(k_predict_by_id, dim3(grid_for(g->n)), dim3(T), 0, s, (const float *)feat.as<float>(), g->n, k,
                       (const uint64_t *)g->optr, (const uint32_t *)g->rank2id, (const float *)g->mlp, dev_pred,
                       dev_feat);
    KC_HIP(hipGetLastError());
    KC_TRY(kc_sync(s));
    return KC_OK;
}

extern "C" kc_status kc_mlp_step(float *dev_params, float *dev_adam_m, float *dev_adam_v, int32_t step, float lr,
                                 const float *dev_x, const float *dev_t, uint32_t count, float *dev_grad, float *loss,
                                 void *hip_stream) {
    if (!dev_params || !dev_adam_m || !dev_adam_v || !dev_x || !dev_t) return kc_fail(KC_EINVAL, "NULL argument");
    if (count == 0) return kc_fail(KC_EINVAL, "count must be positive");
    if (step < 1) return kc_fail(KC_EINVAL, "step must be at least 1");
    if (!(lr > 0.f) || lr != lr || lr > 1e30f) return kc_fail(KC_EINVAL, "lr must be positive and finite");
    hipStream_t s = (hipStream_t)hip_stream;
    kc_tmp grad, lsum;
    KC_TRY(kc_tmp_alloc(grad, NP * 4, s));
    KC_TRY(kc_tmp_alloc(lsum, 4, s));
    KC_HIP(hipMemsetAsync(grad.p, 0, NP * 4, s));
    KC_HIP(hipMemsetAsync(lsum.p, 0, 4, s));
    hipLaunchKernelGGL(k_mlp_grad, dim3((count + GB - 1) / GB), dim3(GB), 0, s, dev_x, dev_t, (const uint32_t *)nullptr,
                       (size_t)0, (size_t)count, (const float *)dev_params, grad.as<float>(), lsum.as<float>());
    if (dev_grad) KC_HIP(hipMemcpyAsync(dev_grad, grad.p, NP * 4, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_adam, dim3(1), dim3(256), 0, s, dev_params, grad.as<float>(), dev_adam_m, dev_adam_v, step,
                       lr);
    KC_HIP(hipGetLastError());
    float *h = (float *)kc_pinned_scratch();
    if (loss) KC_HIP(hipMemcpyAsync(h, lsum.p, 4, hipMemcpyDeviceToHost, s));
    KC_TRY(kc_sync(s));
    if (loss) *loss = h[0] / (float)count;
    return KC_OK;
}

extern "C" kc_status kc_set_schedule(kc_graph *g, int32_t policy, const char *weights_path) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (policy != KC_SCHED_DEGREE && policy != KC_SCHED_LEARNED && policy != KC_SCHED_EDGES)
        return kc_fail(KC_EINVAL, "unknown policy %d", policy);
    if (policy == KC_SCHED_LEARNED && weights_path) {
        FILE *f = fopen(weights_path, "rb");
        if (!f) return kc_fail(KC_EINVAL, "cannot open %s", weights_path);
        char magic[8];
        uint32_t np = 0;
        std::vector<float> buf(NP + NORM);
        const bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "KCMLP001", 8) == 0 &&
                        fread(&np, 4, 1, f) == 1 && np == (uint32_t)NP &&
                        fread(buf.data() + NP, 4, NORM, f) == (size_t)NORM && fread(buf.data(), 4, NP, f) == (size_t)NP;
        fclose(f);
        if (!ok) return kc_fail(KC_EINVAL, "%s is not a scheduler weight file", weights_path);
        if (!g->mlp) KC_TRY(kc_dev_alloc((void **)&g->mlp, (NP + NORM) * 4, g->stream));
        KC_HIP(hipMemcpyAsync(g->mlp, buf.data(), (NP + NORM) * 4, hipMemcpyHostToDevice, g->stream));
        KC_TRY(kc_sync(g->stream));
        g->mlp_loaded = 1;
        ++g->mlp_serial;  // learned queues built with other weights are stale
    }
    if (policy == KC_SCHED_LEARNED && !g->mlp_loaded) return kc_fail(KC_ESTATE, "no scheduler weights loaded");
    g->policy = policy;
    return KC_OK;
}

extern "C" kc_status kc_train_schedule(kc_graph *const *gs, uint32_t num, int32_t k, int32_t epochs, uint64_t seed,
                                       const char *weights_path, float *final_loss) {
    if (!gs || num == 0 || !weights_path) return kc_fail(KC_EINVAL, "NULL argument");
    if (k < 4 || k > KC_KMAX) return kc_fail(KC_EINVAL, "k=%d outside [4, %d]", k, KC_KMAX);
    if (epochs < 1) return kc_fail(KC_EINVAL, "epochs must be positive");
    for (uint32_t i = 0; i < num; ++i) {
        if (!gs[i]) return kc_fail(KC_EINVAL, "graph %u is NULL", i);
        if (!gs[i]->oriented) return kc_fail(KC_ESTATE, "graph %u is not oriented", i);
    }
    hipStream_t s = gs[0]->stream;
    // 1. samples (features, log1p work) of every active root, for k' = 4..k
    std::vector<float> hX, hT;
    for (uint32_t gi = 0; gi < num; ++gi) {
        const kc_graph *g = gs[gi];
        for (int kk = 4; kk <= k; ++kk) {
            kc_tmp counts, work, feat, flag, pos, X, Tv, tot;
            KC_TRY(kc_tmp_alloc(counts, (size_t)g->n * 8, g->stream));
            KC_TRY(kc_tmp_alloc(work, (size_t)g->n * 8, g->stream));
            KC_TRY(kc_count_per_root(g, kk, counts.as<uint64_t>(), work.as<uint64_t>()));
            KC_TRY(kc_tmp_alloc(feat, (size_t)g->n * NF * 4, g->stream));
            KC_TRY(features(g, kk, feat.as<float>(), g->stream));
            KC_TRY(kc_tmp_alloc(flag, (size_t)g->n * 4, g->stream));
            KC_TRY(kc_tmp_alloc(pos, (size_t)g->n * 4, g->stream));
            KC_TRY(kc_tmp_alloc(tot, 4, g->stream));
            hipLaunchKernelGGL(k_active_flags, dim3(grid_for(g->n)), dim3(T), 0, g->stream, (const uint64_t *)g->optr,
                               g->n, kk, flag.as<uint32_t>());
            KC_TRY(kc_scan_excl_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), g->n, tot.as<uint32_t>(), g->stream));
            uint32_t na = 0;
            KC_HIP(hipMemcpyAsync(&na, tot.p, 4, hipMemcpyDeviceToHost, g->stream));
            KC_TRY(kc_sync(g->stream));
            if (na == 0) continue;
            KC_TRY(kc_tmp_alloc(X, (size_t)na * NF * 4, g->stream));
            KC_TRY(kc_tmp_alloc(Tv, (size_t)na * 4, g->stream));
            hipLaunchKernelGGL(k_gather, dim3(grid_for(g->n)), dim3(T), 0, g->stream, (const float *)feat.as<float>(),
                               (const uint64_t *)g->optr, (const uint32_t *)g->rank2id,
                               (const uint64_t *)work.as<uint64_t>(), g->n, kk, (const uint32_t *)pos.as<uint32_t>(),
                               X.as<float>(), Tv.as<float>());
            KC_HIP(hipGetLastError());
            const size_t o = hT.size();
            hX.resize(hX.size() + (size_t)na * NF);
            hT.resize(o + na);
            KC_HIP(hipMemcpyAsync(hX.data() + o * NF, X.p, (size_t)na * NF * 4, hipMemcpyDeviceToHost, g->stream));
            KC_HIP(hipMemcpyAsync(hT.data() + o, Tv.p, (size_t)na * 4, hipMemcpyDeviceToHost, g->stream));
            KC_TRY(kc_sync(g->stream));
        }
    }
    const size_t N = hT.size();
    if (N == 0) return kc_fail(KC_EINVAL, "no training samples");
    // 2. standardise features and labels (statistics kept in the weight file)
    std::vector<float> norm(NORM);
    for (int i = 0; i < NF; ++i) {
        double s1 = 0, s2 = 0;
        for (size_t r = 0; r < N; ++r) {
            s1 += hX[r * NF + i];
            s2 += (double)hX[r * NF + i] * hX[r * NF + i];
        }
        const double mu = s1 / N, var = s2 / N - mu * mu;
        norm[i] = (float)mu;
        norm[NF + i] = (float)(var > 1e-12 ? sqrt(var) : 1.0);
    }
    {
        double s1 = 0, s2 = 0;
        for (size_t r = 0; r < N; ++r) {
            s1 += hT[r];
            s2 += (double)hT[r] * hT[r];
        }
        const double mu = s1 / N, var = s2 / N - mu * mu;
        norm[2 * NF] = (float)mu;
        norm[2 * NF + 1] = (float)(var > 1e-12 ? sqrt(var) : 1.0);
    }
    for (size_t r = 0; r < N; ++r) {
        for (int i = 0; i < NF; ++i) hX[r * NF + i] = (hX[r * NF + i] - norm[i]) / norm[NF + i];
        hT[r] = (hT[r] - norm[2 * NF]) / norm[2 * NF + 1];
    }
    // 3. seeded initialisation (uniform, He-scaled) and a seeded sample order
    std::vector<float> hp(NP, 0.f);
    uint64_t st = seed;
    auto u01 = [&st]() {
        st = kc_mix64(st);
        return (float)((st >> 11) * 0x1.0p-53);
    };
    for (int i = 0; i < NF * H; ++i) hp[OFF_W1 + i] = (2.f * u01() - 1.f) * sqrtf(6.f / NF);
    for (int i = 0; i < H * H; ++i) hp[OFF_W2 + i] = (2.f * u01() - 1.f) * sqrtf(6.f / H);
    for (int i = 0; i < H; ++i) hp[OFF_W3 + i] = (2.f * u01() - 1.f) * sqrtf(3.f / H);
    std::vector<uint32_t> order(N);
    for (size_t r = 0; r < N; ++r) order[r] = (uint32_t)r;
    for (size_t r = N - 1; r > 0; --r) {
        st = kc_mix64(st);
        const size_t j = (size_t)(((st >> 32) * (uint64_t)(r + 1)) >> 32);
        const uint32_t tmp = order[r];
        order[r] = order[j];
        order[j] = tmp;
    }
    kc_tmp dX, dT, dO, dP, dG, dM, dV, dL;
    KC_TRY(kc_tmp_alloc(dX, N * NF * 4, s));
    KC_TRY(kc_tmp_alloc(dT, N * 4, s));
    KC_TRY(kc_tmp_alloc(dO, N * 4, s));
    KC_TRY(kc_tmp_alloc(dP, NP * 4, s));
    KC_TRY(kc_tmp_alloc(dG, NP * 4, s));
    KC_TRY(kc_tmp_alloc(dM, NP * 4, s));
    KC_TRY(kc_tmp_alloc(dV, NP * 4, s));
    KC_TRY(kc_tmp_alloc(dL, 4, s));
    KC_HIP(hipMemcpyAsync(dX.p, hX.data(), N * NF * 4, hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(dT.p, hT.data(), N * 4, hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(dO.p, order.data(), N * 4, hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(dP.p, hp.data(), NP * 4, hipMemcpyHostToDevice, s));
    KC_HIP(hipMemsetAsync(dG.p, 0, NP * 4, s));
    KC_HIP(hipMemsetAsync(dM.p, 0, NP * 4, s));
    KC_HIP(hipMemsetAsync(dV.p, 0, NP * 4, s));
    // 4. mini-batch Adam
    const size_t B = 4096;
    int step = 0;
    float loss = 0.f;
    for (int ep = 0; ep < epochs; ++ep) {
        KC_HIP(hipMemsetAsync(dL.p, 0, 4, s));
        for (size_t b0 = 0; b0 < N; b0 += B) {
            const size_t cnt = (N - b0) < B ? (N - b0) : B;
            hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((cnt + GB - 1) / GB)), dim3(GB), 0, s,
                               (const float *)dX.as<float>(), (const float *)dT.as<float>(),
                               (const uint32_t *)dO.as<uint32_t>(), b0, cnt, (const float *)dP.as<float>(),
                               dG.as<float>(), dL.as<float>());
            ++step;
            hipLaunchKernelGGL(k_adam, dim3(1), dim3(256), 0, s, dP.as<float>(), dG.as<float>(), dM.as<float>(),
                               dV.as<float>(), step, 2e-3f);
        }
        KC_HIP(hipGetLastError());
        KC_HIP(hipMemcpyAsync(&loss, dL.p, 4, hipMemcpyDeviceToHost, s));
        KC_TRY(kc_sync(s));
        loss /= (float)N;  // mean over the epoch's samples of 0.5 (y - t)^2, each at its batch's parameters
    }
    KC_HIP(hipMemcpyAsync(hp.data(), dP.p, NP * 4, hipMemcpyDeviceToHost, s));
    KC_TRY(kc_sync(s));
    FILE *f = fopen(weights_path, "wb");
    if (!f) return kc_fail(KC_EINVAL, "cannot write %s", weights_path);
    const uint32_t np = NP;
    const bool ok = fwrite("KCMLP001", 1, 8, f) == 8 && fwrite(&np, 4, 1, f) == 1 &&
                    fwrite(norm.data(), 4, NORM, f) == (size_t)NORM && fwrite(hp.data(), 4, NP, f) == (size_t)NP;
    fclose(f);
    if (!ok) return kc_fail(KC_EDEVICE, "short write to %s", weights_path);
    if (final_loss) *final_loss = loss;
    return KC_OK;
}
