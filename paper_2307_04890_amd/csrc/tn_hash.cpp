// C ABI of network hashing (Sec. 4.1) and fusion (Sec. 4.2).
#include <algorithm>
#include <vector>

#include "tn_batch.h"
#include "tn_hash.h"

namespace {
constexpr uint64_t kP61 = (1ull << 61) - 1;
constexpr size_t kLiftedBudget = (size_t)1 << 30;  // bytes of lifted tables per pass
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

extern "C" {

tn_status tn_hash_compress(tn_ctx *ctx, uint32_t n, int64_t m, const uint32_t *src,
                           const uint32_t *dst, const int64_t *t, uint32_t flags, uint32_t H,
                           uint32_t K, const uint64_t *coeffs, int32_t order, uint32_t *bucket,
                           int32_t *count, tn_batch **proxies) {
    using namespace tn;
    if (!ctx || !proxies) return fail(TN_E_ARG, "ctx or proxies is NULL");
    *proxies = nullptr;
    if (n == 0 || H == 0 || K == 0 || order < 1) return fail(TN_E_ARG, "n, H, K and order must be > 0");
    if (K > 65536) return fail(TN_E_UNSUPPORTED, "K must be <= 65536");
    if (!coeffs || !bucket || !count) return fail(TN_E_ARG, "null coefficient or output array");
    for (size_t i = 0; i < (size_t)H * 3 * order; ++i)
        if (coeffs[i] >= kP61) return fail(TN_E_ARG, "hash coefficients must be < 2^61 - 1");
    if (m < 0 || (m > 0 && (!src || !dst || !t))) return fail(TN_E_ARG, "bad event arrays");
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] >= n || dst[e] >= n) return fail(TN_E_RANGE, "event " + std::to_string(e) + " has a node id >= n");
        if (e > 0 && t[e] < t[e - 1]) return fail(TN_E_ORDER, "event " + std::to_string(e) + " is earlier than its predecessor");
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    const size_t cbytes = sizeof(uint64_t) * H * 3 * order;
    tn_status st = ensure_scratch(ctx, cbytes);
    if (st != TN_OK) return st;
    hipError_t e = hipMemcpyAsync(ctx->scratch, coeffs, cbytes, hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "coefficient upload");
    {
        ProfScope ps(ctx, TN_K_HASH);
        e = launch_hash_buckets(n, H, (const uint64_t *)ctx->scratch, order, K, bucket, count,
                                ctx->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "hash kernel launch");
    // the host planner needs the bucket map of every hash
    std::vector<uint32_t> hb((size_t)H * n);
    e = hipMemcpyAsync(hb.data(), bucket, sizeof(uint32_t) * hb.size(), hipMemcpyDeviceToHost,
                       ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "bucket download");
    std::vector<uint32_t> ns(H, K);
    std::vector<int64_t> ms(H, m);
    std::vector<const uint32_t *> ss(H, src), ds(H, dst), maps(H);
    std::vector<const int64_t *> ts(H, t);
    for (uint32_t j = 0; j < H; ++j) maps[j] = hb.data() + (size_t)j * n;
    return batch_create(ctx, (int32_t)H, ns.data(), ms.data(), ss.data(), ds.data(), ts.data(),
                        flags, proxies, maps.data(), n);
}

tn_status tn_recombine(tn_ctx *ctx, uint32_t n, uint32_t H, uint32_t K, const uint64_t *P,
                       int64_t ldK, const uint32_t *bucket, const int32_t *count, int32_t *est,
                       int32_t *lifted) {
    using namespace tn;
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    if (n == 0 || H == 0 || K == 0) return fail(TN_E_ARG, "n, H and K must be > 0");
    if (K > 65536) return fail(TN_E_UNSUPPORTED, "K must be <= 65536");
    if (ldK < (int64_t)((K + 63) / 64)) return fail(TN_E_ARG, "ldK must be >= ceil(K/64)");
    if (!P || !bucket || !count || !est) return fail(TN_E_ARG, "null device array");
    if (recombine_group(K) == 0) return fail(TN_E_UNSUPPORTED, "K too large for the LDS tables");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    const uint32_t nq = (n + 63) / 64;
    const size_t per_q = (size_t)H * K * 8;
    uint32_t qr = (uint32_t)std::max<size_t>(4, std::min<size_t>(nq, kLiftedBudget / per_q));
    qr = (qr + 3) / 4 * 4;
    const size_t pt_bytes = align256((size_t)H * K * ldK * 8);
    const size_t rs_bytes = align256((size_t)H * K * 4);
    const size_t full_bytes = align256((size_t)H * K);
    const size_t list_bytes = align256((size_t)n * 4 + 4);
    const size_t lt_bytes = align256((size_t)qr * per_q);
    tn_status st = ensure_scratch(ctx, pt_bytes + rs_bytes + full_bytes + list_bytes + lt_bytes);
    if (st != TN_OK) return st;
    unsigned char *base = (unsigned char *)ctx->scratch;
    uint64_t *PT = (uint64_t *)base;
    int32_t *rowsum = (int32_t *)(base + pt_bytes);
    uint8_t *full = base + pt_bytes + rs_bytes;
    uint32_t *list = (uint32_t *)(base + pt_bytes + rs_bytes + full_bytes);
    uint32_t *nlist_dev = list + n;
    uint64_t *Lt = (uint64_t *)(base + pt_bytes + rs_bytes + full_bytes + list_bytes);
    hipError_t e;
    uint32_t nlist = 0;
    {
        ProfScope ps(ctx, TN_K_AUX);
        e = launch_transpose_proxies(H, K, ldK, P, PT, ctx->stream);
        if (e == hipSuccess && lifted)
            e = launch_lifted_sizes(n, H, K, ldK, P, bucket, count, rowsum, lifted, ctx->stream);
        if (e == hipSuccess)
            e = launch_split_full(n, H, K, ldK, P, bucket, full, est, list, nlist_dev, ctx->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(&nlist, nlist_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "recombine set-up kernels");
    for (uint32_t q0 = 0; nlist > 0 && q0 < nq; q0 += qr) {
        const uint32_t cnt = std::min(qr, nq - q0);
        {
            ProfScope ps(ctx, TN_K_AUX);
            e = launch_build_lifted(n, H, K, ldK, PT, bucket, q0, cnt, Lt, ctx->stream);
        }
        if (e != hipSuccess) return hip_fail(e, "lifted-table kernel launch");
        {
            ProfScope ps(ctx, TN_K_RECOMBINE);
            e = launch_recombine_est(n, H, K, bucket, Lt, q0, cnt, list, nlist, est, ctx->stream);
        }
        if (e != hipSuccess) return hip_fail(e, "recombine kernel launch");
    }
    return TN_OK;
}

}  // extern "C"
