// Batched counting: placeholder loop until the persistent batch kernel lands.
#include "kc_internal.h"

extern "C" kc_status kc_count_batch(kc_graph *const *gs, uint32_t num, int32_t k, uint64_t *q_out) {
    if (!gs || !q_out) return kc_fail(KC_EINVAL, "NULL argument");
    for (uint32_t i = 0; i < num; ++i) KC_TRY(kc_count(gs[i], k, &q_out[i]));
    return KC_OK;
}
