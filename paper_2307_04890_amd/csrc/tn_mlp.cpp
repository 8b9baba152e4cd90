// C ABI of the learned combiner.
#include <cmath>

#include "tn_mlp.h"

extern "C" {

int32_t tn_mlp_param_count(void) { return tn::mlp_param_count(); }

tn_status tn_mlp_init(tn_ctx *ctx, uint64_t seed, float *params) {
    using namespace tn;
    if (!ctx || !params) return fail(TN_E_ARG, "null argument");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    hipError_t e;
    {
        ProfScope ps(ctx, TN_K_AUX);
        e = launch_mlp_init(seed, params, ctx->stream);
    }
    return e == hipSuccess ? TN_OK : hip_fail(e, "init kernel launch");
}

tn_status tn_mlp_features(tn_ctx *ctx, uint32_t n, uint32_t H, const int32_t *lifted, float *x) {
    using namespace tn;
    if (!ctx || !lifted || !x) return fail(TN_E_ARG, "null argument");
    if (n == 0) return fail(TN_E_ARG, "n must be > 0");
    if (H != 16) return fail(TN_E_UNSUPPORTED, "the combiner takes H = 16 lifted sizes");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    hipError_t e;
    {
        ProfScope ps(ctx, TN_K_AUX);
        e = launch_mlp_features(n, H, lifted, x, ctx->stream);
    }
    return e == hipSuccess ? TN_OK : hip_fail(e, "feature kernel launch");
}

tn_status tn_mlp_forward(tn_ctx *ctx, const float *params, const float *x, int64_t N, float *yhat) {
    using namespace tn;
    if (!ctx || !params || !x || !yhat) return fail(TN_E_ARG, "null argument");
    if (N < 0) return fail(TN_E_ARG, "N must be >= 0");
    if (N > (int64_t)1 << 37) return fail(TN_E_UNSUPPORTED, "N too large");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    hipError_t e;
    {
        ProfScope ps(ctx, TN_K_MLP_FORWARD);
        e = launch_mlp_forward(params, x, N, yhat, ctx->stream);
    }
    return e == hipSuccess ? TN_OK : hip_fail(e, "forward kernel launch");
}

tn_status tn_mlp_predict(tn_ctx *ctx, const float *params, const float *x, int64_t N,
                         uint32_t n_nodes, const int32_t *est, float *sizes) {
    using namespace tn;
    if (!ctx || !params || !x || !sizes) return fail(TN_E_ARG, "null argument");
    if (N < 0 || n_nodes == 0) return fail(TN_E_ARG, "N must be >= 0 and n_nodes > 0");
    if (N > (int64_t)1 << 37) return fail(TN_E_UNSUPPORTED, "N too large");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    hipError_t e;
    {
        ProfScope ps(ctx, TN_K_MLP_FORWARD);
        e = launch_mlp_predict(params, x, N, n_nodes, est, sizes, ctx->stream);
    }
    return e == hipSuccess ? TN_OK : hip_fail(e, "predict kernel launch");
}

tn_status tn_mlp_train_step(tn_ctx *ctx, float *params, float *adam_m, float *adam_v, int64_t step,
                            const float *x, const float *y, const int32_t *idx, int64_t N, float lr,
                            float *loss, float *grad) {
    using namespace tn;
    if (!ctx || !params || !adam_m || !adam_v || !x || !y) return fail(TN_E_ARG, "null argument");
    if (N <= 0) return fail(TN_E_ARG, "N must be > 0");
    if (N > ((int64_t)1 << 31) - 1) return fail(TN_E_UNSUPPORTED, "N must be < 2^31");
    if (step < 1) return fail(TN_E_ARG, "step is 1-based");
    if (!(lr > 0.f)) return fail(TN_E_ARG, "lr must be > 0");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    const int nblk = mlp_backward_blocks(N);
    const size_t need = sizeof(float) * ((size_t)nblk * mlp_param_count() + nblk);
    tn_status st = ensure_scratch(ctx, need);
    if (st != TN_OK) return st;
    float *partial = (float *)ctx->scratch;
    float *loss_partial = partial + (size_t)nblk * mlp_param_count();
    // Adam bias corrections 1 / (1 - beta^step)
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)step)));
    hipError_t e;
    {
        ProfScope ps(ctx, TN_K_MLP_BACKWARD);
        e = launch_mlp_backward(params, x, y, idx, N, partial, loss_partial, ctx->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "backward kernel launch");
    {
        ProfScope ps(ctx, TN_K_MLP_ADAM);
        e = launch_mlp_adam(partial, nblk, params, adam_m, adam_v, lr, c1, c2, loss_partial, loss,
                            grad, ctx->stream);
    }
    return e == hipSuccess ? TN_OK : hip_fail(e, "Adam kernel launch");
}

}  // extern "C"
