// Batched counting: many graphs in one persistent launch sequence.
//
// The batch is laid out on the device as one disjoint union: graph i's ranks are
// shifted by the nodes of graphs 0..i-1, so its out-lists, and hence every G+(u),
// are unchanged.  One queue holds the roots of all graphs, ordered by tier, then
// graph, then out-degree (heaviest first), so that a wave's partial sum changes
// graph rarely; the tier kernels add each graph's cliques to that graph's total.
// The count launches are captured once in a HIP graph and replayed when the same
// handles are counted again at the same k.  Tunables come from kc_set_tuning or
// from the autotuner below, which times the batch over a grid of them.
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "kc_internal.h"

namespace {

constexpr int T = 256;
inline unsigned grid_for(size_t n) { return (unsigned)((n + T - 1) / T); }

__global__ void k_concat(const uint64_t *optr, const uint32_t *ocol, uint32_t n, uint64_t m, uint32_t nbase,
                         uint64_t mbase, uint32_t gid, uint64_t *optr_b, uint32_t *ocol_b, uint32_t *graph_of) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        optr_b[nbase + i] = optr[i] + mbase;
        graph_of[nbase + i] = gid;
    }
    if (i < m) ocol_b[mbase + i] = ocol[i] + nbase;
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) { *p = v; }

// key = tier (2 bits: scratch 0, workgroup 1, wave 2) | graph | out-degree complement | rank
__global__ void k_batch_keys(const uint64_t *optr, const uint32_t *graph_of, uint32_t n, int k, uint32_t wd,
                             uint32_t dcap, int gbits, uint64_t *keys, uint32_t *flag, uint32_t *stats) {
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool active = false;
    uint32_t tier = 0, d = 0;
    if (u < n) {
        d = (uint32_t)(optr[u + 1] - optr[u]);
        active = d >= (uint32_t)(k - 1);
        tier = d > dcap ? 0u : (d > wd ? 1u : 2u);
        const int dbits = 30 - gbits;
        const uint32_t dmaxv = (1u << dbits) - 1u;
        const uint32_t dc = d < dmaxv ? d : dmaxv;
        const uint64_t hi = ((uint64_t)tier << 30) | ((uint64_t)graph_of[u] << dbits) | (uint64_t)(dmaxv - dc);
        keys[u] = (hi << 32) | (uint64_t)u;
        flag[u] = active ? 1u : 0u;
    }
#pragma unroll
    for (uint32_t t = 0; t < 3; ++t) {
        const bool in = active && tier == t;
        const uint32_t c = (uint32_t)__popcll(__ballot(in));
        const uint32_t m = kc_wave_max_u32(in ? d : 0u);
        if ((threadIdx.x & 63) == 0 && c) {
            atomicAdd(&stats[t], c);
            atomicMax(&stats[4 + t], m);
        }
    }
}

__global__ void k_compact(const uint64_t *keys, const uint32_t *flag, const uint32_t *pos, uint32_t n, uint64_t *out) {
    const size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n && flag[u]) out[pos[u]] = keys[u];
}

__global__ void k_low32(const uint64_t *keys, uint32_t cnt, uint32_t *q) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) q[i] = (uint32_t)keys[i];
}

struct Plan {
    std::vector<uint64_t> key;  // handle serials, k, tunables
    kc_graph bg;                // the disjoint union (owns optr/ocol through kc_tmp below)
    kc_tmp optr, ocol, graph_of, gtot, res, queue, gscr;
    kc_tmp lrows, wbits, woff;  // the queued roots' staged G+(u) (see kc_stage_queue)
    bool cached = false;
    kc_queue q;
    size_t slice_words = 0;
    uint32_t scratch_blocks = 0;
    uint32_t num = 0;
    int k = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool eager_only = false;  // capture unavailable (default stream, or capture failed)
    ~Plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};
std::mutex g_plan_mu;
Plan *g_plan = nullptr;

std::vector<uint64_t> plan_key(kc_graph *const *gs, uint32_t num, int k) {
    const kc_tuning_t &tu = kc_tuning_now();
    std::vector<uint64_t> key;
    key.reserve(num + 6);
    for (uint32_t i = 0; i < num; ++i) key.push_back(gs[i]->serial);
    key.push_back((uint64_t)k);
    key.push_back((uint64_t)tu.wave_dmax);
    key.push_back((uint64_t)tu.wg_blocks_per_cu);
    key.push_back((uint64_t)tu.wave_blocks_per_cu);
    key.push_back((uint64_t)tu.chunk_div);
    key.push_back((uint64_t)tu.wg_dmax);
    key.push_back((uint64_t)tu.local_bits);
    key.push_back((uint64_t)tu.wg_waves);
    return key;
}

kc_status build_plan(kc_graph *const *gs, uint32_t num, int k, Plan &P) {
    hipStream_t s = gs[0]->stream;
    uint64_t N = 0, M = 0;
    for (uint32_t i = 0; i < num; ++i) {
        N += gs[i]->n;
        M += gs[i]->m;
    }
    if (N >= (1ull << 32) || M >= (1ull << 32)) return kc_fail(KC_EINVAL, "batch too large (%llu nodes)", (unsigned long long)N);
    kc_graph &bg = P.bg;
    bg.device = gs[0]->device;
    bg.stream = s;
    bg.n = (uint32_t)N;
    bg.m = M;
    bg.oriented = 1;
    KC_TRY(kc_tmp_alloc(P.optr, (N + 1) * 8, s));
    KC_TRY(kc_tmp_alloc(P.ocol, (M ? M : 1) * 4, s));
    KC_TRY(kc_tmp_alloc(P.graph_of, (N ? N : 1) * 4, s));
    KC_TRY(kc_tmp_alloc(P.gtot, (size_t)num * 8, s));
    KC_TRY(kc_tmp_alloc(P.res, KC_RES_WORDS * 8, s));
    bg.optr = P.optr.as<uint64_t>();
    bg.ocol = P.ocol.as<uint32_t>();
    bg.rank2id = nullptr;  // exact totals only: ids are never read
    uint64_t nb = 0, mb = 0;
    uint32_t dmax = 0;
    for (uint32_t i = 0; i < num; ++i) {
        const kc_graph *g = gs[i];
        const size_t work = g->n > g->m ? g->n : g->m;
        if (work)
            hipLaunchKernelGGL(k_concat, dim3(grid_for(work)), dim3(T), 0, s, (const uint64_t *)g->optr,
                               (const uint32_t *)g->ocol, g->n, g->m, (uint32_t)nb, mb, i, bg.optr, bg.ocol,
                               P.graph_of.as<uint32_t>());
        nb += g->n;
        mb += g->m;
        dmax = g->max_outdeg > dmax ? g->max_outdeg : dmax;
    }
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, bg.optr + N, (uint64_t)M);
    KC_HIP(hipGetLastError());
    bg.max_outdeg = dmax;

    // queue: tier, graph, out-degree
    const uint32_t dcap = kc_lds_dcap(bg.device, k);
    int wd = kc_tuning_now().wave_dmax;
    wd = wd < 1 ? 1 : (wd > 64 ? 64 : wd);
    int gbits = 1;
    while ((1u << gbits) < num) ++gbits;
    kc_tmp keys, flag, pos, stats, keys2, tmp;
    KC_TRY(kc_tmp_alloc(keys, (N ? N : 1) * 8, s));
    KC_TRY(kc_tmp_alloc(flag, (N ? N : 1) * 4, s));
    KC_TRY(kc_tmp_alloc(pos, (N ? N : 1) * 4, s));
    KC_TRY(kc_tmp_alloc(stats, 8 * 4, s));
    KC_HIP(hipMemsetAsync(stats.p, 0, 8 * 4, s));
    if (N)
        hipLaunchKernelGGL(k_batch_keys, dim3(grid_for(N)), dim3(T), 0, s, (const uint64_t *)bg.optr,
                           (const uint32_t *)P.graph_of.as<uint32_t>(), (uint32_t)N, k, (uint32_t)wd, dcap, gbits,
                           keys.as<uint64_t>(), flag.as<uint32_t>(), stats.as<uint32_t>());
    KC_HIP(hipGetLastError());
    KC_TRY(kc_scan_excl_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), N, nullptr, s));
    uint32_t *h = (uint32_t *)kc_pinned_scratch();
    KC_HIP(hipMemcpyAsync(h, stats.p, 8 * 4, hipMemcpyDeviceToHost, s));
    KC_TRY(kc_sync(s));
    // key tiers: 0 scratch, 1 workgroup, 2 wave  ->  kc_queue tiers 2, 1, 0
    const uint32_t cs = h[0], cw = h[1], cv = h[2], total = cs + cw + cv;
    P.q.count[2] = cs;
    P.q.count[1] = cw;
    P.q.count[0] = cv;
    P.q.max_d[2] = h[4];
    P.q.max_d[1] = h[5];
    P.q.max_d[0] = h[6];
    KC_TRY(kc_tmp_alloc(P.queue, (size_t)(total ? total : 1) * 4, s));
    if (total) {
        KC_TRY(kc_tmp_alloc(keys2, (size_t)total * 8, s));
        KC_TRY(kc_tmp_alloc(tmp, (size_t)total * 8, s));
        hipLaunchKernelGGL(k_compact, dim3(grid_for(N)), dim3(T), 0, s, (const uint64_t *)keys.as<uint64_t>(),
                           (const uint32_t *)flag.as<uint32_t>(), (const uint32_t *)pos.as<uint32_t>(), (uint32_t)N,
                           keys2.as<uint64_t>());
        KC_TRY(kc_radix_sort_u64(keys2.as<uint64_t>(), tmp.as<uint64_t>(), total, 32, 64, s));
        hipLaunchKernelGGL(k_low32, dim3(grid_for(total)), dim3(T), 0, s, (const uint64_t *)keys2.as<uint64_t>(),
                           total, P.queue.as<uint32_t>());
        KC_HIP(hipGetLastError());
    }
    const uint32_t *qb = P.queue.as<uint32_t>();
    P.q.ptr[2] = qb;
    P.q.ptr[1] = qb + cs;
    P.q.ptr[0] = qb + cs + cw;
    KC_TRY(kc_count_scratch(&bg, P.q, k, P.gscr, P.slice_words, P.scratch_blocks));
    P.num = num;
    P.k = k;
    // stage the queued roots' G+(u) once: every run of the plan counts from them
    const char *sc = getenv("KC_STAGE_CACHE");
    if (!(sc && sc[0] == '0')) {
        KC_TRY(kc_stage_queue(&bg, P.q, wd, P.res.as<uint64_t>(), P.lrows, P.wbits, P.woff, P.cached));
    }
    bg.stage_wd = wd;
    bg.lrows = P.cached ? P.lrows.as<uint64_t>() : nullptr;
    bg.wbits = P.cached ? P.wbits.as<uint64_t>() : nullptr;
    bg.woff = P.cached ? P.woff.as<uint64_t>() : nullptr;
    return KC_OK;
}

kc_status run_plan(Plan &P, uint64_t *q_out) {
    hipStream_t s = P.bg.stream;
    kc_count_args a;
    a.k = P.k;
    a.cached = P.cached ? 1 : 0;
    if (!P.exec) {
        // first run eagerly (it also sets kernel attributes), then capture for replays
        KC_TRY(kc_count_launch(&P.bg, P.q, a, P.res.as<uint64_t>(), (unsigned long long *)P.gtot.p, P.num,
                               P.graph_of.as<uint32_t>(), P.gscr.as<uint64_t>(), P.slice_words, P.scratch_blocks, s));
        if (s && !P.eager_only) {
            KC_TRY(kc_sync(s));
            bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
            kc_status st = KC_OK;
            if (ok)
                st = kc_count_launch(&P.bg, P.q, a, P.res.as<uint64_t>(), (unsigned long long *)P.gtot.p, P.num,
                                     P.graph_of.as<uint32_t>(), P.gscr.as<uint64_t>(), P.slice_words,
                                     P.scratch_blocks, s);
            hipGraph_t gr = nullptr;
            if (ok) ok = hipStreamEndCapture(s, &gr) == hipSuccess && st == KC_OK && gr;
            if (ok) ok = hipGraphInstantiate(&P.exec, gr, nullptr, nullptr, 0) == hipSuccess;
            if (getenv("KC_DEBUG")) fprintf(stderr, "[kc] batch of %u graphs, k=%d: count launches %s\n", P.num, P.k,
                                            ok ? "captured in a HIP graph" : "not capturable, replayed eagerly");
            if (ok) {
                P.graph = gr;
            } else {
                // replays fall back to eager launches of the same kernels
                if (gr) (void)hipGraphDestroy(gr);
                P.exec = nullptr;
                P.eager_only = true;
                (void)hipGetLastError();
            }
        }
    } else {
        KC_HIP(hipGraphLaunch(P.exec, s));
    }

    uint64_t *res = kc_pinned_scratch();
    KC_HIP(hipMemcpyAsync(q_out, P.gtot.p, (size_t)P.num * 8, hipMemcpyDeviceToHost, s));
    KC_HIP(hipMemcpyAsync(res, P.res.p, 16, hipMemcpyDeviceToHost, s));
    KC_TRY(kc_sync(s));
    if (res[1]) return kc_fail(KC_EOVERFLOW, "a graph's count does not fit in 64 bits");
    return KC_OK;
}

kc_status batch_impl(kc_graph *const *gs, uint32_t num, int32_t k, uint64_t *q_out) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    std::vector<uint64_t> key = plan_key(gs, num, k);
    if (!g_plan || g_plan->key != key) {
        delete g_plan;
        g_plan = nullptr;
        Plan *P = new (std::nothrow) Plan();
        if (!P) return kc_fail(KC_ENOMEM, "batch plan");
        kc_status st = build_plan(gs, num, k, *P);
        if (st != KC_OK) {
            (void)kc_sync(gs[0]->stream);
            delete P;
            return st;
        }
        P->key = key;
        g_plan = P;
    }
    return run_plan(*g_plan, q_out);
}

kc_status check_batch(kc_graph *const *gs, uint32_t num, int32_t k) {
    if (!gs) return kc_fail(KC_EINVAL, "gs is NULL");
    if (num == 0 || num > 65536) return kc_fail(KC_EINVAL, "num=%u outside [1, 65536]", num);
    if (k < 3 || k > KC_KMAX) return kc_fail(KC_EINVAL, "k=%d outside [3, %d]", k, KC_KMAX);
    for (uint32_t i = 0; i < num; ++i) {
        if (!gs[i]) return kc_fail(KC_EINVAL, "graph %u is NULL", i);
        if (!gs[i]->oriented) return kc_fail(KC_ESTATE, "graph %u is not oriented", i);
        if (gs[i]->stream != gs[0]->stream || gs[i]->device != gs[0]->device)
            return kc_fail(KC_EINVAL, "graphs of one batch must share the device and the stream");
    }
    return KC_OK;
}

std::string arch_name(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

}  // namespace

extern "C" kc_status kc_count_batch(kc_graph *const *gs, uint32_t num, int32_t k, uint64_t *q_out) {
    if (!q_out) return kc_fail(KC_EINVAL, "q_out is NULL");
    KC_TRY(check_batch(gs, num, k));
    return batch_impl(gs, num, k, q_out);
}

// Destroying a handle must drop a cached plan that refers to it.
void kc_batch_forget(uint64_t serial) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (!g_plan) return;
    for (size_t i = 0; i < g_plan->num; ++i)  // the key starts with the handles' serials
        if (g_plan->key[i] == serial) {
            (void)kc_sync(g_plan->bg.stream);
            delete g_plan;
            g_plan = nullptr;
            return;
        }
}

extern "C" kc_status kc_autotune(kc_graph *const *gs, uint32_t num, int32_t k, const char *cache_path, kc_tuning *best) {
    KC_TRY(check_batch(gs, num, k));
    uint64_t N = 0, M = 0;
    for (uint32_t i = 0; i < num; ++i) {
        N += gs[i]->n;
        M += gs[i]->m;
    }
    char keybuf[256];
    snprintf(keybuf, sizeof(keybuf), "%s|graphs=%u|n=%llu|m=%llu|k=%d", arch_name(gs[0]->device).c_str(), num,
             (unsigned long long)N, (unsigned long long)M, k);
    const std::string key = keybuf;
    // cache: one entry per line, "key\twave_dmax wg_blocks wave_blocks chunk_div wg_dmax local_bits wg_waves seconds"
    std::vector<std::string> lines;
    if (cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char line[512];
            while (fgets(line, sizeof(line), f)) {
                std::string l(line);
                while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
                if (l.empty()) continue;
                lines.push_back(l);
                const size_t tab = l.find('\t');
                if (tab != std::string::npos && l.substr(0, tab) == key) {
                    kc_tuning t;
                    double sec = 0;
                    if (sscanf(l.c_str() + tab + 1, "%d %d %d %d %d %d %d %lf", &t.wave_dmax, &t.wg_blocks_per_cu,
                               &t.wave_blocks_per_cu, &t.queue_chunk_div, &t.wg_dmax, &t.local_bits, &t.wg_waves,
                               &sec) == 8) {
                        fclose(f);
                        KC_TRY(kc_set_tuning(&t));
                        if (best) *best = t;
                        return KC_OK;
                    }
                }
            }
            fclose(f);
        }
    }
    std::vector<uint64_t> out(num);
    // bin thresholds (the one-wave tier's out-degree limit), workgroup blocks per CU,
    // wave blocks per CU, queue chunk divisor and the local-graph tile width
    const int wds[] = {24, 48, 64};
    const int wgb[] = {0, 2};
    const int wvb[] = {4, 8};
    const int cds[] = {4, 16};
    const int lbs[] = {64, 128};
    kc_tuning bt{64, 0, 8, 8, 0, 128, 0};
    double bsec = 1e30;
    for (int a : wds)
        for (int b : wgb)
            for (int c : wvb)
                for (int d : cds)
                    for (int e : lbs) {
                        if (k < 6 && e != 64) continue;  // two-word local graphs serve k >= 6 only
                        kc_tuning t{a, b, c, d, 0, e, 0};
                        KC_TRY(kc_set_tuning(&t));
                        KC_TRY(kc_count_batch(gs, num, k, out.data()));  // builds, runs eagerly and captures
                        const int reps = 3;
                        const auto t0 = std::chrono::steady_clock::now();
                        for (int r = 0; r < reps; ++r) KC_TRY(kc_count_batch(gs, num, k, out.data()));
                        const double sec =
                            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() / reps;
                        if (sec < bsec) {
                            bsec = sec;
                            bt = t;
                        }
                    }
    KC_TRY(kc_set_tuning(&bt));
    if (best) *best = bt;
    if (cache_path) {
        FILE *f = fopen(cache_path, "w");
        if (!f) return kc_fail(KC_EINVAL, "cannot write %s", cache_path);
        for (const std::string &l : lines)
            if (l.substr(0, l.find('\t')) != key) fprintf(f, "%s\n", l.c_str());
        fprintf(f, "%s\t%d %d %d %d %d %d %d %.9f\n", key.c_str(), bt.wave_dmax, bt.wg_blocks_per_cu,
                bt.wave_blocks_per_cu, bt.queue_chunk_div, bt.wg_dmax, bt.local_bits, bt.wg_waves, bsec);
        fclose(f);
    }
    return KC_OK;
}
