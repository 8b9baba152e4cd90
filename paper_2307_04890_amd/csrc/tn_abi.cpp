// C ABI: context, plans, validation and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "tn_internal.h"
#include "tn_mlp.h"
#include "tn_wave.h"

namespace {
thread_local std::string g_err;
}  // namespace

namespace tn {
tn_status fail(tn_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

tn_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return TN_E_HIP;
}
}  // namespace tn

using tn::DeviceGuard;
using tn::fail;
using tn::hip_fail;

namespace tn {
tn_status not_built(const char *what) {
    return fail(TN_E_UNSUPPORTED, std::string(what) + " is not built in this library version");
}

// Grows the context scratch to at least `bytes` (waits for the stream first,
// since queued kernels may still use the old buffer).
tn_status ensure_scratch(tn_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->scratch_bytes) return TN_OK;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
    e = hipMalloc(&ctx->scratch, want);
    if (e != hipSuccess) {
        ctx->scratch = nullptr;
        return fail(TN_E_NOMEM, "scratch allocation of " + std::to_string(want) + " bytes failed");
    }
    ctx->scratch_bytes = want;
    return TN_OK;
}

tn_status ensure_host_staging(tn_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->host_staging_bytes) return TN_OK;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (ctx->host_staging) (void)hipHostFree(ctx->host_staging);
    tn::ring_free(ctx);
    ctx->host_staging = nullptr;
    ctx->host_staging_bytes = 0;
    e = hipHostMalloc(&ctx->host_staging, bytes, 0);
    if (e != hipSuccess) {
        ctx->host_staging = nullptr;
        return fail(TN_E_NOMEM, "pinned staging allocation of " + std::to_string(bytes) + " bytes failed");
    }
    ctx->host_staging_bytes = bytes;
    return TN_OK;
}
}  // namespace tn

extern "C" {

const char *tn_last_error(void) { return g_err.c_str(); }

tn_status tn_create(int device, void *stream, tn_ctx **out) {
    if (!out) return fail(TN_E_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(TN_E_ARG, "no such device");
    tn_ctx *c = new (std::nothrow) tn_ctx();
    if (!c) return fail(TN_E_NOMEM, "context allocation failed");
    c->device = device;
    c->stream = (hipStream_t)stream;
    {
        DeviceGuard g(device);
        if (hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess)
            c->num_cus = 256;
        // the static scratch of tn_mlp_train_step_noalloc on this device
        e = g.ok ? tn::mlp_noalloc_bind(device) : hipErrorInvalidDevice;
    }
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "binding the static training scratch");
    }
    *out = c;
    return TN_OK;
}

tn_status tn_set_stream(tn_ctx *ctx, void *stream) {
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    ctx->stream = (hipStream_t)stream;
    return TN_OK;
}

tn_status tn_sync(tn_ctx *ctx) {
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return TN_OK;
}

void tn_destroy(tn_ctx *ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->host_staging) (void)hipHostFree(ctx->host_staging);
    tn::ring_free(ctx);
    if (ctx->traffic) (void)hipFree(ctx->traffic);
    for (auto &r : ctx->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    delete ctx;
}

tn_status tn_profile_enable(tn_ctx *ctx, int enable) {
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    ctx->profiling = enable != 0;
    return TN_OK;
}

int32_t tn_profile_take(tn_ctx *ctx, int32_t *ids, float *ms, int32_t cap) {
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    if (cap < 0 || (cap > 0 && (!ids || !ms))) return fail(TN_E_ARG, "bad output arrays");
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int32_t k = 0;
    for (auto &r : ctx->recs) {
        if (k < cap) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, r.a, r.b);
            ids[k] = r.id;
            ms[k] = (e == hipSuccess) ? t : -1.f;
            ++k;
        }
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    return k;
}

tn_status tn_plan_create(tn_ctx *ctx, uint32_t n, int64_t m, const uint32_t *src,
                         const uint32_t *dst, const int64_t *t, uint32_t flags,
                         tn_plan **out) {
    if (!ctx || !out) return fail(TN_E_ARG, "ctx or out is NULL");
    *out = nullptr;
    tn::HostSchedule hs;
    std::string err;
    const bool hll = flags & TN_HLL;
    tn_status st = tn::plan_events(n, m, src, dst, t, flags & ~(uint32_t)TN_HLL, hs, err, nullptr,
                                   0, hll ? tn::kFormGather : tn::kFormOps);
    if (st != TN_OK) return fail(st, err);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    tn_plan *p = new (std::nothrow) tn_plan();
    if (!p) return fail(TN_E_NOMEM, "plan allocation failed");
    p->device = ctx->device;
    p->hll = hll;
    std::vector<unsigned char> img;
    if (hll) tn::schedule_pack(hs, img);
    else tn::ops_pack(hs, img);
    // a small network with short levels also keeps its ops in the flat form
    const int64_t nops = (int64_t)(hs.ops.size() / 4);
    const bool flat = !hll && tn::rowor_wave_pays(n, hs.scratch_rows, nops, hs.Lops) &&
                      !tn::rowor_wave_wide(nops, hs.Lops);
    const size_t flat_off = (img.size() + 255) & ~(size_t)255;
    if (flat) {
        img.resize(flat_off + tn::flat_ops_bytes(hs), 0);
        tn::flat_ops_pack(hs, n, (uint32_t *)(img.data() + flat_off));
    }
    p->dev_bytes = img.size();
    hipError_t e = hipMalloc(&p->dev, p->dev_bytes);
    if (e != hipSuccess) {
        delete p;
        return fail(TN_E_NOMEM, "device schedule allocation failed");
    }
    e = hipMemcpyAsync(p->dev, img.data(), img.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(p->dev);
        delete p;
        return hip_fail(e, "schedule upload");
    }
    tn::fill_stats(hs, p->stats);
    if (hll) {
        p->gview = tn::schedule_view(hs, p->dev);
        p->lvl_pair = std::move(hs.lvl_pair);
        p->lvl_gat = std::move(hs.lvl_gat);
    } else {
        p->view = tn::ops_view(hs, p->dev);
        if (flat) p->flat = (const uint32_t *)((unsigned char *)p->dev + flat_off);
        p->scratch_rows = hs.scratch_rows;
        p->zero_levels = tn::zero_phase_levels(hs, n);
        {
            // the saturating path's forwarding phase ends where the ops reach
            // kFwdPhaseOpsPerNode * n
            uint32_t l = p->zero_levels;
            while (l < hs.Lops && (int64_t)hs.lvl_op[l] < tn::kFwdPhaseOpsPerNode * (int64_t)n) ++l;
            p->mid_end = l;
        }
        p->host_lvl_op = std::move(hs.lvl_op);
        p->host_ops = std::move(hs.ops);
    }
    *out = p;
    return TN_OK;
}

}  // extern "C"

namespace tn {
void fill_stats(const HostSchedule &hs, tn_plan_stats &s) {
    s.n = hs.n;
    s.m = hs.m;
    const bool ops_only = hs.L == 0 && !hs.lvl_op.empty();
    if (ops_only) {
        s.levels = hs.Lops;
        s.pairs = hs.op_pairs;
        s.gathers = hs.op_targets;
        s.gather_sources = hs.op_sources;
        s.compound_items = hs.op_compound;
        s.directed_pairs = hs.op_directed;
        s.max_level_gathers = 0;
        int64_t widest = 0;
        for (size_t l = 0; l + 1 < hs.lvl_op.size(); ++l)
            widest = std::max<int64_t>(widest, hs.lvl_op[l + 1] - hs.lvl_op[l]);
        s.max_level_items = widest;
        s.device_bytes = (int64_t)ops_device_bytes(hs);
    } else {
        s.levels = hs.L;
        s.pairs = (int64_t)hs.pairs.size() / 2;
        s.gathers = (int64_t)hs.gat_tgt.size();
        s.gather_sources = (int64_t)hs.gat_src.size();
        s.compound_items = hs.compound_items;
        s.directed_pairs = hs.directed_pairs;
        s.max_level_items = hs.max_level_items;
        s.max_level_gathers = hs.max_level_gathers;
        s.device_bytes = (int64_t)schedule_device_bytes(hs);
    }
    s.host_seconds = hs.host_seconds;
    s.ops = (int64_t)hs.ops.size() / 4;
    s.op_levels = hs.Lops;
    s.scratch_rows = hs.scratch_rows;
}
}  // namespace tn

extern "C" {

struct tn_host_schedule {
    tn::HostSchedule hs;
    std::vector<uint32_t> flvl, fops;  // the forwarded op form, made on request
    uint32_t fcap = 0;                 // ... with levels of at most this many ops
};

tn_status tn_schedule_build(uint32_t n, int64_t m, const uint32_t *src, const uint32_t *dst,
                            const int64_t *t, uint32_t flags, tn_host_schedule **out) {
    if (!out) return fail(TN_E_ARG, "out is NULL");
    *out = nullptr;
    tn_host_schedule *s = new (std::nothrow) tn_host_schedule();
    if (!s) return fail(TN_E_NOMEM, "schedule allocation failed");
    std::string err;
    tn_status st = tn::plan_events(n, m, src, dst, t, flags, s->hs, err, nullptr, 0,
                                   tn::kFormGather | tn::kFormOps);
    if (st != TN_OK) {
        delete s;
        return fail(st, err);
    }
    *out = s;
    return TN_OK;
}

tn_status tn_schedule_arrays(const tn_host_schedule *s, tn_plan_stats *stats,
                             const uint32_t **lvl_pair, const uint32_t **lvl_gat,
                             const uint32_t **pairs, const uint32_t **gat_tgt,
                             const uint32_t **gat_ptr, const uint32_t **gat_src) {
    if (!s) return fail(TN_E_ARG, "schedule is NULL");
    if (stats) tn::fill_stats(s->hs, *stats);
    if (lvl_pair) *lvl_pair = s->hs.lvl_pair.data();
    if (lvl_gat) *lvl_gat = s->hs.lvl_gat.data();
    if (pairs) *pairs = s->hs.pairs.data();
    if (gat_tgt) *gat_tgt = s->hs.gat_tgt.data();
    if (gat_ptr) *gat_ptr = s->hs.gat_ptr.data();
    if (gat_src) *gat_src = s->hs.gat_src.data();
    return TN_OK;
}

tn_status tn_schedule_op_arrays(const tn_host_schedule *s, const uint32_t **lvl_op,
                                const uint32_t **ops) {
    if (!s) return fail(TN_E_ARG, "schedule is NULL");
    if (lvl_op) *lvl_op = s->hs.lvl_op.data();
    if (ops) *ops = s->hs.ops.data();
    return TN_OK;
}

tn_status tn_schedule_fwd_arrays(tn_host_schedule *s, uint32_t level_cap, uint32_t *levels,
                                 const uint32_t **lvl, const uint32_t **ops) {
    if (!s || !levels) return fail(TN_E_ARG, "schedule or levels is NULL");
    if (level_cap == 0 || level_cap > tn::kFwdLevelCap) level_cap = tn::kFwdLevelCap;
    if (s->flvl.empty() || s->fcap != level_cap) {
        tn::fwd_schedule(s->hs.lvl_op, s->hs.ops, s->hs.n, s->hs.scratch_rows, level_cap, s->flvl,
                         s->fops);
        s->fcap = level_cap;
    }
    *levels = (uint32_t)s->flvl.size() - 1;
    if (lvl) *lvl = s->flvl.data();
    if (ops) *ops = s->fops.data();
    return TN_OK;
}

void tn_schedule_destroy(tn_host_schedule *s) { delete s; }

tn_status tn_plan_get_stats(const tn_plan *plan, tn_plan_stats *out) {
    if (!plan || !out) return fail(TN_E_ARG, "plan or out is NULL");
    *out = plan->stats;
    return TN_OK;
}

void tn_plan_destroy(tn_plan *plan) {
    if (!plan) return;
    DeviceGuard g(plan->device);
    for (auto x : plan->hll_execs) (void)hipGraphExecDestroy(x);
    if (plan->fwd_dev) (void)hipFree(plan->fwd_dev);
    if (plan->mid_dev) (void)hipFree(plan->mid_dev);
    if (plan->dev) (void)hipFree(plan->dev);
    delete plan;
}

int64_t tn_recommended_ld(uint32_t n) {
    const int64_t nwords = ((int64_t)n + 63) / 64;
    return nwords >= 16 ? (nwords + 15) / 16 * 16 : nwords;
}

namespace {
// A forwarded schedule of the plan's op levels [l0, l1) on the device,
// made on first use (waits for the upload): the whole plan for the plain
// recurrence, the middle range for the saturating path's forwarding phase.
tn_status plan_fwd(tn_ctx *ctx, const tn_plan *plan, uint32_t l0, uint32_t l1, void **dev,
                   tn::DevOps *view) {
    std::lock_guard<std::mutex> lk(plan->fwd_mu);
    if (*dev) return TN_OK;
    std::vector<uint32_t> lvl, ops;
    const std::vector<uint32_t> &hl = plan->host_lvl_op;
    for (uint32_t l = l0; l <= l1; ++l) lvl.push_back(hl[l] - hl[l0]);
    ops.assign(plan->host_ops.begin() + 4 * (size_t)hl[l0], plan->host_ops.begin() + 4 * (size_t)hl[l1]);
    std::vector<uint32_t> flvl, fops;
    tn::fwd_schedule(lvl, ops, plan->stats.n, plan->scratch_rows, tn::kFwdLevelCap, flvl, fops);
    const size_t lb = (4 * flvl.size() + 255) & ~(size_t)255;
    const size_t bytes = lb + 4 * std::max<size_t>(fops.size(), 4);
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return fail(TN_E_NOMEM, "forwarded schedule allocation failed");
    e = hipMemcpyAsync(d, flvl.data(), 4 * flvl.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess && !fops.empty())
        e = hipMemcpyAsync((unsigned char *)d + lb, fops.data(), 4 * fops.size(),
                           hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "forwarded schedule upload");
    }
    view->L = (uint32_t)flvl.size() - 1;
    view->nops = (uint32_t)(fops.size() / 4);
    view->lvl = (const uint32_t *)d;
    view->ops = (const uint4 *)((unsigned char *)d + lb);
    *dev = d;
    return TN_OK;
}
}  // namespace

tn_status tn_plan_execute(tn_ctx *ctx, const tn_plan *plan, uint64_t *C, int64_t ld,
                          uint32_t slice_words) {
    if (!ctx || !plan) return fail(TN_E_ARG, "ctx or plan is NULL");
    if (!C) return fail(TN_E_ARG, "C is NULL");
    const uint32_t n = plan->stats.n;
    const int64_t nwords = (n + 63) / 64;
    if (ld < nwords) return fail(TN_E_ARG, "ld must be >= ceil(n/64)");
    if (plan->device != ctx->device) return fail(TN_E_ARG, "plan lives on another device");
    if (plan->hll) return fail(TN_E_ARG, "a TN_HLL plan runs only tn_hll_execute");
    // a small network with the slice width left to the library runs on one
    // wavefront per word column, its column in LDS
    const bool wave = slice_words == 0 && tn::default_slice_words(n, ld) == 1 &&
                      tn::rowor_wave_pays(n, plan->scratch_rows, plan->stats.ops,
                                          plan->stats.op_levels);
    if (slice_words == 0) slice_words = tn::default_slice_words(n, ld);
    if (slice_words > 64 || (slice_words & (slice_words - 1)))
        return fail(TN_E_ARG, "slice_words must be a power of two <= 64");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    // per-workgroup sink words (for the widest grid of the launches below,
    // so that every launch finds the compound scratch rows at one place),
    // then those rows, then (for a zero phase) the slice state the launches
    // share, its done counter and the slice order of the last launch
    const uint32_t tail_sw = tn::tail_slice_words(n, slice_words, ctx->num_cus);
    const uint32_t sinks = tn::rowor_workgroups(n, tail_sw);
    const size_t sink_rows_words =
        (size_t)sinks * tn::kRoworSinkWords +
        (size_t)plan->scratch_rows * (size_t)tn::scratch_stride((uint32_t)nwords);
    const bool zero_phase = !wave && ctx->saturation && plan->zero_levels > 0;
    const size_t pwords = zero_phase ? tn::rowor_persist_words(n, tail_sw) + 1 : 0;
    const size_t owords = zero_phase ? sinks : 0;
    {
        tn_status st = tn::ensure_scratch(ctx, sizeof(uint64_t) * sink_rows_words +
                                                   4 * (pwords + owords));
        if (st != TN_OK) return st;
    }
    uint32_t *persist = zero_phase ? (uint32_t *)((uint64_t *)ctx->scratch + sink_rows_words) : nullptr;
    uint32_t *order = zero_phase ? persist + pwords : nullptr;
    ctx->state = nullptr;
    ctx->state_sw = 0;
    hipError_t e;
    if (!ctx->traffic) {
        e = hipMalloc((void **)&ctx->traffic, 2 * sizeof(unsigned long long));
        if (e != hipSuccess) {
            ctx->traffic = nullptr;
            return fail(TN_E_NOMEM, "traffic counter allocation failed");
        }
    }
    {
        tn::ProfScope ps(ctx, TN_K_IDENTITY);
        e = tn::launch_identity(C, n, ld, ctx->traffic, ctx->stream);
        if (e == hipSuccess && persist)
            e = tn::launch_fill_u32(persist, pwords, 0u, ctx->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "identity kernel launch");
    // the plain recurrence (saturation off, or no room for its bitmap) runs
    // on the forwarded schedule where the slice width allows
    const bool fwd = !wave && (!ctx->saturation || !tn::rowor_saturates(n, plan->scratch_rows)) &&
                     tn::rowor_fwd_supported(n, slice_words) && plan->stats.ops > 0;
    if (fwd) {
        tn_status st = plan_fwd(ctx, plan, 0, plan->stats.op_levels, &plan->fwd_dev,
                                &plan->fwd_view);
        if (st != TN_OK) return st;
    }
    // the saturating path of a large network: the zero phase, then the
    // forwarding kernel while most ops still move rows, then the per-slice
    // state rebuilt from the matrix and the saturating kernel for the rest
    const bool three = !fwd && zero_phase && n >= 16384 && tn::rowor_saturates(n, plan->scratch_rows) &&
                       tn::rowor_fwd_supported(n, slice_words) &&
                       plan->mid_end > plan->zero_levels && plan->mid_end < plan->stats.op_levels;
    if (three) {
        tn_status st = plan_fwd(ctx, plan, plan->zero_levels, plan->mid_end, &plan->mid_dev,
                                &plan->mid_view);
        if (st != TN_OK) return st;
    }
    {
        tn::ProfScope ps(ctx, TN_K_ROWOR);
        if (fwd) {
            e = tn::launch_rowor_fwd(plan->fwd_view, n, C, ld, slice_words,
                                     (uint64_t *)ctx->scratch, sinks, plan->scratch_rows,
                                     ctx->traffic, ctx->stream);
        } else if (three) {
            tn::DevOps head = plan->view, tail = plan->view;
            head.L = plan->zero_levels;
            tail.L = plan->view.L - plan->mid_end;
            tail.lvl = plan->view.lvl + plan->mid_end;
            unsigned int *done = persist + pwords - 1;
            e = tn::launch_rowor_global(head, n, C, ld, slice_words, (uint64_t *)ctx->scratch,
                                        sinks, plan->scratch_rows, ctx->traffic, true, persist,
                                        done, plan->zero_levels, nullptr, ctx->stream);
            if (e == hipSuccess)
                e = tn::launch_rowor_fwd(plan->mid_view, n, C, ld, slice_words,
                                         (uint64_t *)ctx->scratch, sinks, plan->scratch_rows,
                                         ctx->traffic, ctx->stream);
            // the rest on narrower slices, the slices with the most rows
            // still not full first
            if (e == hipSuccess)
                e = tn::launch_slice_full_state(C, ld, n, tail_sw, persist, ctx->stream);
            if (e == hipSuccess) e = tn::launch_slice_order(persist, n, tail_sw, order, ctx->stream);
            if (e == hipSuccess)
                e = tn::launch_rowor_global(tail, n, C, ld, tail_sw, (uint64_t *)ctx->scratch,
                                            sinks, plan->scratch_rows, ctx->traffic, true, persist,
                                            done, 0u, order, ctx->stream);
            if (e == hipSuccess) {
                ctx->state = persist;
                ctx->state_sw = tail_sw;
            }
        } else if (wave && plan->flat)
            e = tn::launch_rowor_wave_flat1(plan->flat, plan->view.nops, n, C, ld,
                                            plan->scratch_rows, ctx->traffic, ctx->saturation,
                                            ctx->stream);
        else if (wave)
            e = tn::launch_rowor_wave(plan->view, n, C, ld, plan->scratch_rows, ctx->traffic,
                                      ctx->saturation, nullptr, nullptr, ctx->stream);
        else {
            e = tn::launch_rowor_global(plan->view, n, C, ld, slice_words,
                                        (uint64_t *)ctx->scratch, sinks, plan->scratch_rows,
                                        ctx->traffic, ctx->saturation, persist,
                                        persist ? persist + pwords - 1 : nullptr,
                                        zero_phase ? plan->zero_levels : 0u, nullptr, ctx->stream);
            // a launch that kept no state (no room for the bitmap) left the
            // zeroed state: no slice counts as done
            if (e == hipSuccess && persist) {
                ctx->state = persist;
                ctx->state_sw = slice_words;
            }
        }
    }
    if (e != hipSuccess) return hip_fail(e, "row-OR kernel launch");
    return TN_OK;
}

tn_status tn_set_saturation(tn_ctx *ctx, int enable) {
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    ctx->saturation = enable != 0;
    return TN_OK;
}

tn_status tn_plan_last_traffic(tn_ctx *ctx, uint64_t *words) {
    if (!ctx || !words) return fail(TN_E_ARG, "ctx or words is NULL");
    words[0] = words[1] = 0;
    if (!ctx->traffic) return TN_OK;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    unsigned long long h[2];
    e = hipMemcpy(h, ctx->traffic, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "traffic counter copy");
    words[0] = h[0];
    words[1] = h[1];
    return TN_OK;
}

tn_status tn_build_component_matrix(tn_ctx *ctx, uint32_t n, int64_t m, const uint32_t *src,
                                    const uint32_t *dst, const int64_t *t, uint32_t flags,
                                    uint64_t *C, int64_t ld) {
    return tn::build_streamed(ctx, n, m, src, dst, t, flags, C, ld, 0, nullptr);
}

}  // extern "C"

namespace {
// The level launches of a TN_HLL plan as a HIP graph (captured on a stream
// of its own, then launched on the context's): one launch per level costs
// the host more than the device, and a graph replays them back to back.
// Captured again when the rows, the scratch or the row width change.
tn_status hll_graph(tn_ctx *ctx, const tn_plan *plan, uint32_t nwords, uint8_t *M,
                    const uint64_t *Grow, unsigned int *left, bool sat) {
    if (plan->gview.L == 0) return TN_OK;
    if (!plan->hll_execs.empty() && plan->hll_M == M && plan->hll_scr == ctx->scratch &&
        plan->hll_nwords == nwords && plan->hll_sat == sat)
        return TN_OK;
    if (!plan->hll_execs.empty()) {
        // a queued replay may still run the old graphs
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        for (auto x : plan->hll_execs) (void)hipGraphExecDestroy(x);
        plan->hll_execs.clear();
    }
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    for (uint32_t l0 = 0; l0 < plan->gview.L && e == hipSuccess; l0 += tn::kHllSegmentLevels) {
        hipGraph_t g = nullptr;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) break;
        hipError_t le = tn::launch_hll_levels(plan->gview, plan->lvl_pair.data(),
                                              plan->lvl_gat.data(), l0,
                                              l0 + tn::kHllSegmentLevels, nwords, (uint64_t *)M,
                                              (uint64_t *)ctx->scratch, sat ? Grow : nullptr,
                                              sat ? left : nullptr, cs);
        e = hipStreamEndCapture(cs, &g);
        if (le != hipSuccess) e = le;
        hipGraphExec_t x = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e == hipSuccess) plan->hll_execs.push_back(x);
        if (g) (void)hipGraphDestroy(g);
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        for (auto x : plan->hll_execs) (void)hipGraphExecDestroy(x);
        plan->hll_execs.clear();
        return hip_fail(e, "HLL level graph");
    }
    plan->hll_M = M;
    plan->hll_scr = ctx->scratch;
    plan->hll_nwords = nwords;
    plan->hll_sat = sat;
    return TN_OK;
}
}  // namespace

extern "C" {

tn_status tn_hll_execute(tn_ctx *ctx, const tn_plan *plan, uint32_t log2s,
                         const uint64_t *node_hash, uint8_t *M, double *est) {
    if (!ctx || !plan) return fail(TN_E_ARG, "ctx or plan is NULL");
    if (!node_hash || !M) return fail(TN_E_ARG, "node_hash or M is NULL");
    if (log2s < 4 || log2s > 16) return fail(TN_E_ARG, "log2s must be in [4, 16]");
    if ((uintptr_t)M % 16 != 0) return fail(TN_E_ARG, "M must start on 16 bytes");
    if (plan->device != ctx->device) return fail(TN_E_ARG, "plan lives on another device");
    const uint32_t n = plan->stats.n;
    const uint32_t nwords = (1u << log2s) / 8;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    // TN_HLL plans: one scratch row per gather of the widest level, then
    // the saturation row G, the count of rows not yet G and 2^log2s uint32
    // for the register maxima; others: per-workgroup sink words, then the
    // compound scratch rows
    const size_t gat_words = (size_t)std::max<uint32_t>(plan->gview.max_gat, 1) * nwords;
    {
        const size_t words =
            plan->hll ? gat_words + nwords + 1 + ((size_t)1 << log2s) / 2
                      : (size_t)tn::rowmax_workgroups(nwords) * tn::kRoworSinkWords +
                            (size_t)plan->scratch_rows *
                                (size_t)tn::scratch_stride((uint32_t)nwords);
        tn_status st = tn::ensure_scratch(ctx, sizeof(uint64_t) * words);
        if (st != TN_OK) return st;
    }
    uint64_t *Grow = (uint64_t *)ctx->scratch + gat_words;
    unsigned int *left = (unsigned int *)(Grow + nwords);
    unsigned int *gmax = (unsigned int *)(Grow + nwords + 1);
    const bool sat = plan->hll && ctx->saturation;
    hipError_t e;
    if (!ctx->traffic) {
        e = hipMalloc((void **)&ctx->traffic, 2 * sizeof(unsigned long long));
        if (e != hipSuccess) {
            ctx->traffic = nullptr;
            return fail(TN_E_NOMEM, "traffic counter allocation failed");
        }
    }
    {
        tn::ProfScope ps(ctx, TN_K_AUX);
        e = tn::launch_fill_u32((uint32_t *)ctx->traffic, 4, 0u, ctx->stream);
        if (e == hipSuccess) e = tn::launch_hll_init(n, log2s, node_hash, M, ctx->stream);
        if (e == hipSuccess && sat)
            e = tn::launch_hll_saturation_setup(n, log2s, node_hash, M, gmax, Grow, left,
                                                ctx->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "HLL init launch");
    {
        if (plan->hll) {
            std::lock_guard<std::mutex> lk(plan->hll_mu);
            tn_status st = hll_graph(ctx, plan, nwords, M, Grow, left, sat);
            if (st != TN_OK) return st;
            unsigned int *snap = nullptr;  // pinned copies of *left, two slots
            hipEvent_t ev[2] = {nullptr, nullptr};
            if (sat && plan->hll_execs.size() > 2) {
                st = tn::ensure_host_staging(ctx, 2 * sizeof(unsigned int));
                if (st != TN_OK) return st;
                snap = (unsigned int *)ctx->host_staging;
                for (int k = 0; k < 2 && e == hipSuccess; ++k)
                    e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
            }
            {
                // segments in order; with saturation, two in flight, and none
                // launched once one has ended with every row equal to G
                tn::ProfScope ps(ctx, TN_K_ROWOR);
                for (size_t k = 0; k < plan->hll_execs.size() && e == hipSuccess; ++k) {
                    if (snap && k >= 2) {
                        e = hipEventSynchronize(ev[k % 2]);
                        if (e != hipSuccess || snap[k % 2] == 0u) break;
                    }
                    e = hipGraphLaunch(plan->hll_execs[k], ctx->stream);
                    if (snap && e == hipSuccess) {
                        e = hipMemcpyAsync(&snap[k % 2], left, sizeof(unsigned int),
                                           hipMemcpyDeviceToHost, ctx->stream);
                        if (e == hipSuccess) e = hipEventRecord(ev[k % 2], ctx->stream);
                    }
                }
            }
            for (int k = 0; k < 2; ++k)
                if (ev[k]) (void)hipEventDestroy(ev[k]);
        } else {
            tn::ProfScope ps(ctx, TN_K_ROWOR);
            e = tn::launch_rowmax_global(plan->view, n, nwords, (uint64_t *)M, nwords,
                                         (uint64_t *)ctx->scratch, plan->scratch_rows,
                                         ctx->traffic, ctx->stream);
        }
    }
    if (e != hipSuccess) return hip_fail(e, "HLL stream launch");
    if (est) {
        tn::ProfScope ps(ctx, TN_K_AUX);
        e = tn::launch_hll_estimate(n, log2s, M, est, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "HLL estimate launch");
    }
    return TN_OK;
}

tn_status tn_hll_build(tn_ctx *ctx, uint32_t n, int64_t m, const uint32_t *src,
                       const uint32_t *dst, const int64_t *t, uint32_t flags, uint32_t log2s,
                       const uint64_t *node_hash, uint8_t *M, double *est) {
    if (!node_hash || !M) return fail(TN_E_ARG, "node_hash or M is NULL");
    if (log2s < 4 || log2s > 16) return fail(TN_E_ARG, "log2s must be in [4, 16]");
    tn_plan *p = nullptr;
    tn_status st = tn_plan_create(ctx, n, m, src, dst, t, flags | TN_HLL, &p);
    if (st != TN_OK) return st;
    st = tn_hll_execute(ctx, p, log2s, node_hash, M, est);
    if (st == TN_OK) {
        DeviceGuard g(ctx->device);
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    tn_plan_destroy(p);
    return st;
}

namespace {
tn_status component_sizes(tn_ctx *ctx, uint32_t n, const uint64_t *C, int64_t ld,
                          int32_t *out_sizes, int32_t *in_sizes, const uint32_t *state,
                          uint32_t state_sw) {
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    if (n == 0) return fail(TN_E_ARG, "n must be > 0");
    if (!C) return fail(TN_E_ARG, "C is NULL");
    if (ld < (int64_t)((n + 63) / 64)) return fail(TN_E_ARG, "ld must be >= ceil(n/64)");
    if (!out_sizes && !in_sizes) return TN_OK;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    if (out_sizes) {
        tn::ProfScope ps(ctx, TN_K_OUT_SIZES);
        hipError_t e = tn::launch_out_sizes(C, n, ld, out_sizes, ctx->stream, state, state_sw);
        if (e != hipSuccess) return hip_fail(e, "out-size kernel launch");
    }
    if (in_sizes) {
        tn::ProfScope ps(ctx, TN_K_IN_SIZES);
        hipError_t e = tn::launch_in_sizes(C, n, ld, in_sizes, ctx->stream, state, state_sw);
        if (e != hipSuccess) return hip_fail(e, "in-size kernel launch");
    }
    return TN_OK;
}
}  // namespace

tn_status tn_component_sizes(tn_ctx *ctx, uint32_t n, const uint64_t *C, int64_t ld,
                             int32_t *out_sizes, int32_t *in_sizes) {
    return component_sizes(ctx, n, C, ld, out_sizes, in_sizes, nullptr, 0);
}

tn_status tn_plan_execute_sizes(tn_ctx *ctx, const tn_plan *plan, uint64_t *C, int64_t ld,
                                uint32_t slice_words, int32_t *out_sizes, int32_t *in_sizes) {
    tn_status st = tn_plan_execute(ctx, plan, C, ld, slice_words);
    if (st != TN_OK) return st;
    // the state the execution just left describes exactly this matrix
    return component_sizes(ctx, plan->stats.n, C, ld, out_sizes, in_sizes, ctx->state,
                           ctx->state_sw);
}

}  // extern "C"
