// Learned scheduler: placeholder until the MLP kernels land.
#include "kc_internal.h"

kc_status kc_predict_work(const kc_graph *g, int k, float *d_pred, hipStream_t s) {
    (void)g; (void)k; (void)d_pred; (void)s;
    return kc_fail(KC_ESTATE, "learned scheduler not available");
}

extern "C" kc_status kc_set_schedule(kc_graph *g, int32_t policy, const char *weights_path) {
    if (!g) return kc_fail(KC_EINVAL, "graph is NULL");
    (void)weights_path;
    if (policy != KC_SCHED_DEGREE) return kc_fail(KC_EINVAL, "unknown policy %d", policy);
    g->policy = policy;
    return KC_OK;
}

extern "C" kc_status kc_train_schedule(kc_graph *const *gs, uint32_t num, int32_t k, int32_t epochs, uint64_t seed,
                                       const char *weights_path, float *final_loss) {
    (void)gs; (void)num; (void)k; (void)epochs; (void)seed; (void)weights_path; (void)final_loss;
    return kc_fail(KC_ESTATE, "learned scheduler not available");
}
