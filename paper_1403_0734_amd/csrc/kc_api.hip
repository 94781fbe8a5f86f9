// The C ABI of libkc: argument checks, handle life cycle, status codes.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "kc_internal.h"

#include <atomic>

namespace {
thread_local char g_msg[512] = {0};
std::atomic<uint64_t> g_serial{1};
kc_tuning_t g_tuning;

inline int bits_for(uint32_t n) {
    int b = 1;
    while (b < 32 && ((uint64_t)1 << b) < (uint64_t)n) ++b;
    return b;
}
}  // namespace

kc_status kc_fail(kc_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return s;
}

kc_status kc_hip_fail(hipError_t e, const char *what, const char *file, int line) {
    const char *f = strrchr(file, '/');
    snprintf(g_msg, sizeof(g_msg), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), f ? f + 1 : file, line);
    if (e == hipErrorOutOfMemory) return KC_ENOMEM;
    return KC_EDEVICE;
}

kc_status kc_tmp_alloc(kc_tmp &t, size_t bytes, hipStream_t s) {
    if (t.p) {
        kc_cache_free(t.p, t.s);
        t.p = nullptr;
    }
    t.s = s;
    return kc_cache_alloc(&t.p, bytes ? bytes : 8, s);
}

const kc_tuning_t &kc_tuning_now() { return g_tuning; }

kc_status kc_dev_alloc(void **p, size_t bytes, hipStream_t s) {
    kc_tmp t;
    KC_TRY(kc_tmp_alloc(t, bytes, s));
    *p = t.p;
    t.p = nullptr;  // ownership moves to the caller
    return KC_OK;
}

void *kc_pinned_buffer(size_t bytes) {
    static thread_local void *buf = nullptr;
    static thread_local size_t cap = 0;
    if (bytes > cap) {
        if (buf) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        if (hipHostMalloc(&buf, c, hipHostMallocDefault) != hipSuccess) return nullptr;
        cap = c;
    }
    return buf;
}

uint64_t *kc_pinned_scratch() {
    static thread_local uint64_t *buf = nullptr;
    if (!buf) {
        if (hipHostMalloc((void **)&buf, 512, hipHostMallocDefault) != hipSuccess) buf = nullptr;
    }
    return buf;
}

extern "C" {

const char *kc_status_str(kc_status s) {
    static thread_local char buf[640];
    const char *name = "unknown status";
    switch (s) {
        case KC_OK: name = "ok"; break;
        case KC_EINVAL: name = "invalid argument"; break;
        case KC_ESTATE: name = "call out of order"; break;
        case KC_ENOMEM: name = "out of memory"; break;
        case KC_EOVERFLOW: name = "count does not fit in 64 bits"; break;
        case KC_EDEVICE: name = "device error"; break;
    }
    if (s != KC_OK && g_msg[0]) snprintf(buf, sizeof(buf), "%s: %s", name, g_msg);
    else snprintf(buf, sizeof(buf), "%s", name);
    return buf;
}

void kc_graph_destroy(kc_graph *g) {
    if (!g) return;
    kc_batch_forget(g->serial);
    void *bufs[] = {g->rowptr, g->col,  g->deg, g->ukeys, g->optr,  g->ocol,  g->rank2id, g->id2rank,
                    g->mlp,    g->d_res, g->dq,  g->tri,   g->lrows, g->wbits, g->woff, g->feat, g->wq, g->wedges, g->wq2};
    for (void *b : bufs)
        kc_cache_free(b, g->stream);
    for (auto &L : g->lq) {
        kc_cache_free(L.queue, g->stream);
        kc_cache_free(L.items, g->stream);
        kc_cache_free(L.items2, g->stream);
    }
    (void)kc_sync(g->stream);
    delete[] g->dq_hist;
    for (hipEvent_t e : g->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : g->sev)
        if (e) (void)hipEventDestroy(e);
    if (g->fork) (void)hipEventDestroy(g->fork);
    if (g->join) (void)hipEventDestroy(g->join);
    if (g->side) (void)hipStreamDestroy(g->side);
    delete g;
}

static kc_status create_impl(const uint32_t *src, const uint32_t *dst, uint64_t m_in, uint32_t n,
                             int32_t src_on_device, void *hip_stream, kc_graph *g) {
    KC_HIP(hipGetDevice(&g->device));
    g->stream = (hipStream_t)hip_stream;
    g->n = n;
    g->m_in = m_in;
    g->idbits = bits_for(n);
    g->serial = g_serial.fetch_add(1);
    for (auto &e : g->ev) KC_HIP(hipEventCreate(&e));
    for (auto &e : g->sev) KC_HIP(hipEventCreate(&e));
    KC_TRY(kc_dev_alloc((void **)&g->d_res, KC_RES_WORDS * sizeof(uint64_t), g->stream));
    if (!kc_pinned_scratch()) return kc_fail(KC_ENOMEM, "pinned host buffer");
    const uint32_t *ds = src, *dd = dst;
    kc_tmp cs, cd;
    if (!src_on_device && m_in) {
        KC_TRY(kc_tmp_alloc(cs, m_in * sizeof(uint32_t), g->stream));
        KC_TRY(kc_tmp_alloc(cd, m_in * sizeof(uint32_t), g->stream));
        KC_HIP(hipMemcpyAsync(cs.p, src, m_in * sizeof(uint32_t), hipMemcpyHostToDevice, g->stream));
        KC_HIP(hipMemcpyAsync(cd.p, dst, m_in * sizeof(uint32_t), hipMemcpyHostToDevice, g->stream));
        ds = cs.as<uint32_t>();
        dd = cd.as<uint32_t>();
    }
    KC_TRY(kc_canonicalise(g, ds, dd));
    KC_TRY(kc_sync(g->stream));
    return KC_OK;
}

kc_status kc_graph_create(const uint32_t *src, const uint32_t *dst, uint64_t m_in, uint32_t n,
                          int32_t src_on_device, void *hip_stream, kc_graph **out) {
    g_msg[0] = 0;
    if (!out) return kc_fail(KC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n == 0) return kc_fail(KC_EINVAL, "n must be positive");
    if (m_in && (!src || !dst)) return kc_fail(KC_EINVAL, "src or dst is NULL");
    if (m_in >= (1ull << 31)) return kc_fail(KC_EINVAL, "m_in must be below 2^31");
    kc_graph *g = new (std::nothrow) kc_graph();
    if (!g) return kc_fail(KC_ENOMEM, "host allocation failed");
    kc_status st = create_impl(src, dst, m_in, n, src_on_device, hip_stream, g);
    if (st != KC_OK) {
        kc_graph_destroy(g);
        return st;
    }
    *out = g;
    return KC_OK;
}

kc_status kc_orient(kc_graph *g) {
    g_msg[0] = 0;
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (g->oriented) return KC_OK;
    return kc_orient_impl(g);
}

static kc_status check_count(const kc_graph *g, int32_t k, int lo) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (k < lo || k > KC_KMAX) return kc_fail(KC_EINVAL, "k=%d outside [%d, %d]", k, lo, KC_KMAX);
    if (!g->oriented) return kc_fail(KC_ESTATE, "kc_orient has not been called");
    return KC_OK;
}

kc_status kc_count(const kc_graph *g, int32_t k, uint64_t *q_out) {
    g_msg[0] = 0;
    if (!q_out) return kc_fail(KC_EINVAL, "q_out is NULL");
    KC_TRY(check_count(g, k, 1));
    if (k == 1) {
        *q_out = g->n;
        return KC_OK;
    }
    if (k == 2) {
        *q_out = g->m;
        return KC_OK;
    }
    kc_count_args a;
    a.k = k;
    a.policy = g->policy;
    uint64_t total = 0;
    int ovf = 0;
    KC_TRY(kc_count_impl(g, a, &total, &ovf));
    if (ovf) return kc_fail(KC_EOVERFLOW, "q_%d >= 2^64", k);
    *q_out = total;
    return KC_OK;
}

kc_status kc_count_colored(const kc_graph *g, int32_t k, uint32_t c, uint64_t seed, int32_t scheme,
                           kc_estimate *out) {
    g_msg[0] = 0;
    if (!out) return kc_fail(KC_EINVAL, "out is NULL");
    KC_TRY(check_count(g, k, 3));
    if (c == 0) return kc_fail(KC_EINVAL, "c must be at least 1");
    if (scheme != KC_COLOR_PER_ROOT && scheme != KC_COLOR_GLOBAL) return kc_fail(KC_EINVAL, "unknown scheme %d", scheme);
    kc_count_args a;
    a.k = k;
    a.colored = 1;
    a.c = c;
    a.seed = seed;
    a.scheme = scheme;
    a.policy = g->policy;
    uint64_t raw = 0;
    int ovf = 0;
    KC_TRY(kc_count_impl(g, a, &raw, &ovf));
    if (ovf) return kc_fail(KC_EOVERFLOW, "raw colour-sampled count >= 2^64");
    const int e = scheme == KC_COLOR_PER_ROOT ? k - 2 : k - 1;
    // raw * c^e exactly in 128 bits when it fits there (raw < 2^64, c^e < 2^(32 e)),
    // else in long double
    long double estd = (long double)raw;
    for (int i = 0; i < e; ++i) estd *= (long double)c;
    unsigned __int128 est = (unsigned __int128)raw;
    int fits128 = 1;
    for (int i = 0; i < e; ++i) {
        if (est != 0 && (unsigned __int128)c > (~(unsigned __int128)0) / est) {
            fits128 = 0;
            break;
        }
        est *= c;
    }
    out->raw = raw;
    out->scale_exponent = e;
    out->estimate = fits128 ? (double)est : (double)estd;
    out->estimate_fits_u64 = (fits128 && (est >> 64) == 0) ? 1 : 0;
    out->estimate_u64 = out->estimate_fits_u64 ? (uint64_t)est : 0;
    return KC_OK;
}

kc_status kc_count_pair_sampled(const kc_graph *g, int32_t k, double p, uint64_t seed, kc_estimate *out) {
    g_msg[0] = 0;
    if (!out) return kc_fail(KC_EINVAL, "out is NULL");
    KC_TRY(check_count(g, k, 3));
    if (!(p > 0.0 && p <= 1.0)) return kc_fail(KC_EINVAL, "p must be in (0, 1]");
    const long double scaled = (long double)p * 4294967296.0L;
    const uint64_t t = scaled >= 4294967296.0L ? (1ull << 32) : (uint64_t)scaled;  // floor(p 2^32)
    if (t == 0) return kc_fail(KC_EINVAL, "p below 2^-32");
    kc_count_args a;
    a.k = k;
    a.sampled = 1;
    a.pair_t = t;
    a.seed = seed;
    a.policy = g->policy;
    uint64_t raw = 0;
    int ovf = 0;
    KC_TRY(kc_count_impl(g, a, &raw, &ovf));
    if (ovf) return kc_fail(KC_EOVERFLOW, "raw pair-sampled count >= 2^64");
    // each k-clique survives with probability (t / 2^32)^e, e = C(k-1, 2)
    const int e = (k - 1) * (k - 2) / 2;
    long double est = (long double)raw;
    for (int i = 0; i < e; ++i) est *= 4294967296.0L / (long double)t;
    out->raw = raw;
    out->scale_exponent = e;
    out->estimate = (double)est;
    out->estimate_fits_u64 = t == (1ull << 32) ? 1 : 0;  // exact only when every pair is kept
    out->estimate_u64 = out->estimate_fits_u64 ? raw : 0;
    return KC_OK;
}

kc_status kc_graph_info(const kc_graph *g, uint32_t *n, uint64_t *m, uint32_t *max_outdeg) {
    g_msg[0] = 0;
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (max_outdeg) *max_outdeg = g->oriented ? g->max_outdeg : 0;
    return KC_OK;
}

kc_status kc_get_csr(const kc_graph *g, uint64_t *row_ptr, uint32_t *col, uint32_t *deg) {
    g_msg[0] = 0;
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    hipStream_t s = g->stream;
    if (row_ptr || col) KC_TRY(kc_build_csr(const_cast<kc_graph *>(g)));
    if (row_ptr) KC_HIP(hipMemcpyAsync(row_ptr, g->rowptr, ((size_t)g->n + 1) * 8, hipMemcpyDeviceToDevice, s));
    if (col && g->m) KC_HIP(hipMemcpyAsync(col, g->col, 2 * (size_t)g->m * 4, hipMemcpyDeviceToDevice, s));
    if (deg) KC_HIP(hipMemcpyAsync(deg, g->deg, (size_t)g->n * 4, hipMemcpyDeviceToDevice, s));
    KC_TRY(kc_sync(s));
    return KC_OK;
}

kc_status kc_get_oriented(const kc_graph *g, uint64_t *optr, uint32_t *ocol, uint32_t *rank2id) {
    g_msg[0] = 0;
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (!g->oriented) return kc_fail(KC_ESTATE, "kc_orient has not been called");
    hipStream_t s = g->stream;
    if (optr) KC_HIP(hipMemcpyAsync(optr, g->optr, ((size_t)g->n + 1) * 8, hipMemcpyDeviceToDevice, s));
    if (ocol && g->m) KC_HIP(hipMemcpyAsync(ocol, g->ocol, (size_t)g->m * 4, hipMemcpyDeviceToDevice, s));
    if (rank2id) KC_HIP(hipMemcpyAsync(rank2id, g->rank2id, (size_t)g->n * 4, hipMemcpyDeviceToDevice, s));
    KC_TRY(kc_sync(s));
    return KC_OK;
}

kc_status kc_set_tuning(const kc_tuning *t) {
    kc_tuning_t v;
    if (t) {
        if (t->wave_dmax < 1 || t->wave_dmax > 64) return kc_fail(KC_EINVAL, "wave_dmax must be in [1, 64]");
        if (t->wg_blocks_per_cu < 0 || t->wg_blocks_per_cu > 8) return kc_fail(KC_EINVAL, "wg_blocks_per_cu in [0, 8]");
        if (t->wave_blocks_per_cu < 1 || t->wave_blocks_per_cu > 16)
            return kc_fail(KC_EINVAL, "wave_blocks_per_cu in [1, 16]");
        if (t->queue_chunk_div < 1 || t->queue_chunk_div > 64) return kc_fail(KC_EINVAL, "queue_chunk_div in [1, 64]");
        if (t->wg_dmax != 0 && (t->wg_dmax < 64 || t->wg_dmax > 65535))
            return kc_fail(KC_EINVAL, "wg_dmax must be 0 or in [64, 65535]");
        if (t->local_bits != 0 && t->local_bits != 64 && t->local_bits != 128)
            return kc_fail(KC_EINVAL, "local_bits must be 0, 64 or 128");
        if (t->wg_waves != 0 && t->wg_waves != 4 && t->wg_waves != 8 && t->wg_waves != 16)
            return kc_fail(KC_EINVAL, "wg_waves must be 0, 4, 8 or 16");
        v.wave_dmax = t->wave_dmax;
        v.wg_blocks_per_cu = t->wg_blocks_per_cu;
        v.wave_blocks_per_cu = t->wave_blocks_per_cu;
        v.chunk_div = t->queue_chunk_div;
        v.wg_dmax = t->wg_dmax;
        v.local_bits = t->local_bits ? t->local_bits : 128;
        v.wg_waves = t->wg_waves;
    }
    g_tuning = v;
    return KC_OK;
}

kc_status kc_get_tuning(kc_tuning *t) {
    if (!t) return kc_fail(KC_EINVAL, "NULL argument");
    t->wave_dmax = g_tuning.wave_dmax;
    t->wg_blocks_per_cu = g_tuning.wg_blocks_per_cu;
    t->wave_blocks_per_cu = g_tuning.wave_blocks_per_cu;
    t->queue_chunk_div = g_tuning.chunk_div;
    t->wg_dmax = g_tuning.wg_dmax;
    t->local_bits = g_tuning.local_bits;
    t->wg_waves = g_tuning.wg_waves;
    return KC_OK;
}

kc_status kc_last_tier_timings(const kc_graph *g, float *ms_wave, float *ms_workgroup, float *ms_scratch) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (ms_wave) *ms_wave = g->t_tier[0];
    if (ms_workgroup) *ms_workgroup = g->t_tier[1];
    if (ms_scratch) *ms_scratch = g->t_tier[2];
    return KC_OK;
}

kc_status kc_last_stage_timings(const kc_graph *g, float *ms_wave, float *ms_workgroup, float *ms_scratch) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (ms_wave) *ms_wave = g->t_stage_tier[0];
    if (ms_workgroup) *ms_workgroup = g->t_stage_tier[1];
    if (ms_scratch) *ms_scratch = g->t_stage_tier[2];
    return KC_OK;
}

kc_status kc_last_timings(const kc_graph *g, float *ms_schedule, float *ms_count, float *ms_total) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    if (ms_schedule) *ms_schedule = g->t_schedule;
    if (ms_count) *ms_count = g->t_count;
    if (ms_total) *ms_total = g->t_total;
    return KC_OK;
}

}  // extern "C"
