// Learned combiner: a 16 -> 64 -> 64 -> 1 ReLU network in FP32 that maps the
// H = 16 per-hash lifted sizes of a node (log-scaled) to an estimate of its
// log out-component size.  Forward, backward and Adam are plain FP32 vector
// code: the layers are tiny, so one wavefront holds 64 samples, keeps the
// weights in LDS and forms the weight gradients as dot products over its
// samples; partial gradients of the workgroups are then summed in a fixed
// order, so a training step is bit-for-bit deterministic.
//
// Parameter layout (5313 floats): W1 (64 x 16, row-major), b1 (64),
// W2 (64 x 64), b2 (64), W3 (1 x 64), b3 (1).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "tn_mlp.h"

namespace tn {

namespace {

constexpr int kIn = 16, kH = 64;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH, kParams = oB3 + 1;
static_assert(kParams == 5313, "parameter count");
constexpr int kSamples = 64;  // samples per workgroup (one per lane)

__device__ __forceinline__ void load_params(const float *__restrict__ p, float *sp) {
    for (int i = threadIdx.x; i < kParams; i += blockDim.x) sp[i] = p[i];
    __syncthreads();
}

// Forward pass of one sample held in registers; returns the output and fills
// h1 (post-ReLU) and z2 (pre-activation of the second layer).
__device__ __forceinline__ float forward_one(const float *sp, const float (&x)[kIn], float (&h1)[kH],
                                             float (&z2)[kH]) {
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float a = sp[oB1 + o];
#pragma unroll
        for (int i = 0; i < kIn; ++i) a = fmaf(sp[oW1 + o * kIn + i], x[i], a);
        h1[o] = fmaxf(a, 0.f);
    }
    float y = sp[oB3];
    for (int o = 0; o < kH; ++o) {
        float a = sp[oB2 + o];
#pragma unroll
        for (int i = 0; i < kH; ++i) a = fmaf(sp[oW2 + o * kH + i], h1[i], a);
        z2[o] = a;
        y = fmaf(sp[oW3 + o], fmaxf(a, 0.f), y);
    }
    return y;
}

__global__ void __launch_bounds__(64)
k_mlp_forward(const float *__restrict__ params, const float *__restrict__ x, int64_t N,
              float *__restrict__ yhat) {
    __shared__ float sp[kParams];
    load_params(params, sp);
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    float xi[kIn], h1[kH], z2[kH];
#pragma unroll
    for (int i = 0; i < kIn; ++i) xi[i] = x[s * kIn + i];
    yhat[s] = forward_one(sp, xi, h1, z2);
}

__global__ void __launch_bounds__(64)
k_mlp_predict(const float *__restrict__ params, const float *__restrict__ x, int64_t N,
              uint32_t n_nodes, const int32_t *__restrict__ est, float *__restrict__ sizes) {
    __shared__ float sp[kParams];
    load_params(params, sp);
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    float xi[kIn], h1[kH], z2[kH];
#pragma unroll
    for (int i = 0; i < kIn; ++i) xi[i] = x[s * kIn + i];
    const float y = forward_one(sp, xi, h1, z2);
    const float hi = est ? (float)est[s] : (float)n_nodes;
    sizes[s] = fminf(fmaxf((float)n_nodes * expf(y), 1.f), hi);
}

// Per-workgroup partial gradients of the mean squared error over its 64
// samples (scaled by 2/N), and its partial loss (sum of squared residuals / N).
__global__ void __launch_bounds__(64)
k_mlp_backward(const float *__restrict__ params, const float *__restrict__ x,
               const float *__restrict__ y, const int32_t *__restrict__ idx, int64_t N,
               float *__restrict__ partial,
               float *__restrict__ loss_partial) {
    __shared__ float sp[kParams];
    __shared__ float sx[kSamples][kIn];
    __shared__ float sh1[kSamples][kH + 1];
    __shared__ float sh2[kSamples][kH + 1];
    __shared__ float sd2[kSamples][kH + 1];
    __shared__ float sd1[kSamples][kH + 1];
    __shared__ float sdy[kSamples];
    __shared__ float sl[kSamples];
    load_params(params, sp);
    const int t = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * kSamples + t;
    const bool valid = s < N;
    const int64_t row = valid ? (idx ? (int64_t)idx[s] : s) : 0;
    float xi[kIn], h1[kH], z2[kH];
#pragma unroll
    for (int i = 0; i < kIn; ++i) xi[i] = valid ? x[row * kIn + i] : 0.f;
    const float out = forward_one(sp, xi, h1, z2);
    const float r = valid ? out - y[row] : 0.f;
    const float inv_n = 1.f / (float)N;
    const float dy = 2.f * r * inv_n;
    sdy[t] = dy;
    sl[t] = r * r * inv_n;
#pragma unroll
    for (int i = 0; i < kIn; ++i) sx[t][i] = xi[i];
    float d2[kH];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        sh1[t][o] = h1[o];
        sh2[t][o] = fmaxf(z2[o], 0.f);
        d2[o] = z2[o] > 0.f ? dy * sp[oW3 + o] : 0.f;
        sd2[t][o] = d2[o];
    }
    for (int i = 0; i < kH; ++i) {
        float a = 0.f;
#pragma unroll
        for (int o = 0; o < kH; ++o) a = fmaf(d2[o], sp[oW2 + o * kH + i], a);
        sd1[t][i] = h1[i] > 0.f ? a : 0.f;
    }
    __syncthreads();
    // weight gradients: each lane owns whole parameters, summing over the
    // samples in order
    float *pg = partial + (size_t)blockIdx.x * kParams;
    for (int p = t; p < kParams; p += blockDim.x) {
        float g = 0.f;
        if (p < oB1) {
            const int o = p / kIn, i = p % kIn;
            for (int q = 0; q < kSamples; ++q) g = fmaf(sd1[q][o], sx[q][i], g);
        } else if (p < oW2) {
            const int o = p - oB1;
            for (int q = 0; q < kSamples; ++q) g += sd1[q][o];
        } else if (p < oB2) {
            const int o = (p - oW2) / kH, i = (p - oW2) % kH;
            for (int q = 0; q < kSamples; ++q) g = fmaf(sd2[q][o], sh1[q][i], g);
        } else if (p < oW3) {
            const int o = p - oB2;
            for (int q = 0; q < kSamples; ++q) g += sd2[q][o];
        } else if (p < oB3) {
            const int o = p - oW3;
            for (int q = 0; q < kSamples; ++q) g = fmaf(sdy[q], sh2[q][o], g);
        } else {
            for (int q = 0; q < kSamples; ++q) g += sdy[q];
        }
        pg[p] = g;
    }
    if (t == 0) {
        float l = 0.f;
        for (int q = 0; q < kSamples; ++q) l += sl[q];
        loss_partial[blockIdx.x] = l;
    }
}

// Sums the partial gradients in workgroup order and applies one Adam step.
__global__ void __launch_bounds__(256)
k_mlp_adam(const float *__restrict__ partial, int nblk, float *__restrict__ params,
           float *__restrict__ m, float *__restrict__ v, float lr, float c1, float c2,
           const float *__restrict__ loss_partial, float *__restrict__ loss,
           float *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss) {
        float l = 0.f;
        for (int b = 0; b < nblk; ++b) l += loss_partial[b];
        loss[0] = l;
    }
    if (p >= kParams) return;
    float g = 0.f;
    for (int b = 0; b < nblk; ++b) g += partial[(size_t)b * kParams + p];
    if (grad) grad[p] = g;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mn = b1 * m[p] + (1.f - b1) * g;
    const float vn = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mn;
    v[p] = vn;
    params[p] -= lr * (mn * c1) / (sqrtf(vn * c2) + eps);
}

// x[u * H + j] = ln(lifted[j * n + u] / n)
__global__ void __launch_bounds__(256)
k_mlp_features(uint32_t n, uint32_t H, const int32_t *__restrict__ lifted, float *__restrict__ x) {
    const size_t total = (size_t)n * H;
    const float inv = 1.f / (float)n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t u = i / H, j = i % H;
        x[i] = logf((float)lifted[j * n + u] * inv);
    }
}

// Seeded initial parameters: He-uniform weights, zero biases.  Weight p of
// the packed vector takes the p-th output of a SplitMix64 generator seeded
// with `seed` (Steele, Lea and Flood, 2014): state seed + (p + 1) * gamma,
// then the generator's output mix.  Each index is computed on its own, so
// the result does not depend on the launch shape.  The top 24 bits give
// u in [0, 1); the weight is (2u - 1) * bound in fp64, rounded to float once.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t p) {
    uint64_t z = seed + (p + 1) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256)
k_mlp_init(uint64_t seed, double bound1, double bound2, double bound3, float *__restrict__ params) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    double bound;
    if (p < oB1) bound = bound1;
    else if (p >= oW2 && p < oB2) bound = bound2;
    else if (p >= oW3 && p < oB3) bound = bound3;
    else {
        params[p] = 0.f;  // a bias
        return;
    }
    const double u = (double)(splitmix64_at(seed, (uint64_t)p) >> 40) * 0x1p-24;
    params[p] = (float)((2.0 * u - 1.0) * bound);
}

}  // namespace

int mlp_param_count() { return kParams; }

hipError_t launch_mlp_forward(const float *params, const float *x, int64_t N, float *yhat,
                              hipStream_t st) {
    if (N <= 0) return hipSuccess;
    const int64_t blocks = (N + 63) / 64;
    hipLaunchKernelGGL(k_mlp_forward, dim3((uint32_t)blocks), dim3(64), 0, st, params, x, N, yhat);
    return hipGetLastError();
}

hipError_t launch_mlp_predict(const float *params, const float *x, int64_t N, uint32_t n_nodes,
                              const int32_t *est, float *sizes, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    const int64_t blocks = (N + 63) / 64;
    hipLaunchKernelGGL(k_mlp_predict, dim3((uint32_t)blocks), dim3(64), 0, st, params, x, N, n_nodes,
                       est, sizes);
    return hipGetLastError();
}

int mlp_backward_blocks(int64_t N) { return (int)((N + kSamples - 1) / kSamples); }

hipError_t launch_mlp_backward(const float *params, const float *x, const float *y,
                               const int32_t *idx, int64_t N, float *partial, float *loss_partial,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_backward, dim3((uint32_t)mlp_backward_blocks(N)), dim3(64), 0, st,
                       params, x, y, idx, N, partial, loss_partial);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const float *partial, int nblk, float *params, float *m, float *v,
                           float lr, float c1, float c2, const float *loss_partial, float *loss,
                           float *grad, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, partial, nblk,
                       params, m, v, lr, c1, c2, loss_partial, loss, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_init(uint64_t seed, float *params, hipStream_t st) {
    // sqrt(6 / fan_in) of each layer, rounded once on the host
    hipLaunchKernelGGL(k_mlp_init, dim3((kParams + 255) / 256), dim3(256), 0, st, seed,
                       std::sqrt(6.0 / kIn), std::sqrt(6.0 / kH), std::sqrt(6.0 / kH), params);
    return hipGetLastError();
}

hipError_t launch_mlp_features(uint32_t n, uint32_t H, const int32_t *lifted, float *x,
                               hipStream_t st) {
    size_t g = ((size_t)n * H + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_mlp_features, dim3((uint32_t)g), dim3(256), 0, st, n, H, lifted, x);
    return hipGetLastError();
}

}  // namespace tn

// ---- training step without allocation --------------------------------------
//
// The partial gradients and losses of one training step live in a file-scope
// device array instead of the context's scratch, so that callers that cannot
// allocate (code under HIP graph capture, serving loops) can train.  Each GPU
// holds its own copy until the process ends.  In host code the array's name
// is only a stand-in for the symbol: its device address is looked up once
// per device (hipGetSymbolAddress, from tn_create) and only that address is
// passed to kernels.  Every partial the Adam kernel reads is written first by
// the backward kernel of the same call, so nothing needs clearing; calls that
// overlap on one GPU share the array and race.
namespace {
constexpr int64_t kNoAllocMaxSamples = 16384;
constexpr int kNoAllocBlocks = (int)(kNoAllocMaxSamples / 64);
static __device__ __align__(256) float scratch[(size_t)kNoAllocBlocks * (5313 + 1)];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

namespace tn {
// Looks up the array's address on the current device (once per device).
hipError_t mlp_noalloc_bind(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    float *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}
}  // namespace tn

extern "C" tn_status tn_mlp_train_step_noalloc(tn_ctx *ctx, float *params, float *adam_m,
                                               float *adam_v, int64_t step, const float *x,
                                               const float *y, const int32_t *idx, int64_t N,
                                               float lr, float *loss, float *grad) {
    using namespace tn;
    if (!ctx || !params || !adam_m || !adam_v || !x || !y) return fail(TN_E_ARG, "null argument");
    if (N <= 0) return fail(TN_E_ARG, "N must be > 0");
    if (N > kNoAllocMaxSamples)
        return fail(TN_E_UNSUPPORTED, "tn_mlp_train_step_noalloc takes at most 16384 samples per step");
    if (step < 1) return fail(TN_E_ARG, "step is 1-based");
    if (!(lr > 0.f)) return fail(TN_E_ARG, "lr must be > 0");
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(TN_E_ARG, "device out of range");
    float *partial;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        partial = g_scratch_ptr[ctx->device];
    }
    if (!partial) return fail(TN_E_HIP, "the static training scratch of this device is not bound");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    const int nblk = mlp_backward_blocks(N);
    static_assert(kParams == 5313, "array size");
    float *loss_partial = partial + (size_t)nblk * kParams;
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

