// Launchers of the learned-combiner kernels (tn_mlp.hip).
#pragma once

#include "tn_internal.h"

namespace tn {

int mlp_param_count();
int mlp_backward_blocks(int64_t N);
hipError_t launch_mlp_predict(const float *params, const float *x, int64_t N, uint32_t n_nodes,
                              const int32_t *est, float *sizes, hipStream_t st);
hipError_t launch_mlp_forward(const float *params, const float *x, int64_t N, float *yhat,
                              hipStream_t st);
hipError_t launch_mlp_backward(const float *params, const float *x, const float *y,
                               const int32_t *idx, int64_t N,
                               float *partial, float *loss_partial, hipStream_t st);
hipError_t launch_mlp_adam(const float *partial, int nblk, float *params, float *m, float *v,
                           float lr, float c1, float c2, const float *loss_partial, float *loss,
                           float *grad, hipStream_t st);
// Binds the static training scratch of tn_mlp_train_step_noalloc on the
// current device (hipGetSymbolAddress, once per device; tn_create calls it).
hipError_t mlp_noalloc_bind(int device);
hipError_t launch_mlp_init(uint64_t seed, float *params, hipStream_t st);
hipError_t launch_mlp_features(uint32_t n, uint32_t H, const int32_t *lifted, float *x,
                               hipStream_t st);

}  // namespace tn
