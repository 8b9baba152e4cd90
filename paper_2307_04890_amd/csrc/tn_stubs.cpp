// Entry points whose kernels are not built yet: they report TN_E_UNSUPPORTED.
#include "tn_internal.h"

namespace tn { tn_status not_built(const char *what); }

extern "C" {
tn_status tn_batch_create(tn_ctx *, int32_t, const uint32_t *, const int64_t *,
                          const uint32_t *const *, const uint32_t *const *,
                          const int64_t *const *, uint32_t, tn_batch **) {
    return tn::not_built("tn_batch_create");
}
tn_status tn_batch_execute(tn_ctx *, tn_batch *, uint64_t *const *, const int64_t *) {
    return tn::not_built("tn_batch_execute");
}
tn_status tn_batch_get_stats(const tn_batch *, tn_plan_stats *, int64_t *, int64_t *) {
    return tn::not_built("tn_batch_get_stats");
}
void tn_batch_destroy(tn_batch *) {}
tn_status tn_build_component_matrix_batched(tn_ctx *, int32_t, const uint32_t *, const int64_t *,
                                            const uint32_t *const *, const uint32_t *const *,
                                            const int64_t *const *, uint32_t, uint64_t *const *,
                                            const int64_t *) {
    return tn::not_built("tn_build_component_matrix_batched");
}
tn_status tn_hash_compress(tn_ctx *, uint32_t, int64_t, const uint32_t *, const uint32_t *,
                           const int64_t *, uint32_t, uint32_t, uint32_t, const uint64_t *,
                           int32_t, uint32_t *, int32_t *, tn_batch **) {
    return tn::not_built("tn_hash_compress");
}
tn_status tn_recombine(tn_ctx *, uint32_t, uint32_t, uint32_t, const uint64_t *, int64_t,
                       const uint32_t *, const int32_t *, int32_t *, int32_t *) {
    return tn::not_built("tn_recombine");
}
int32_t tn_mlp_param_count(void) { return 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1; }
tn_status tn_mlp_features(tn_ctx *, uint32_t, uint32_t, const int32_t *, float *) {
    return tn::not_built("tn_mlp_features");
}
tn_status tn_mlp_forward(tn_ctx *, const float *, const float *, int64_t, float *) {
    return tn::not_built("tn_mlp_forward");
}
tn_status tn_mlp_train_step(tn_ctx *, float *, float *, float *, int64_t, const float *,
                            const float *, int64_t, float, float *, float *) {
    return tn::not_built("tn_mlp_train_step");
}
}
