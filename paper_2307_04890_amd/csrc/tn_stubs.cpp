// Entry points whose kernels are not built yet: they report TN_E_UNSUPPORTED.
#include "tn_internal.h"


extern "C" {
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
