// Host side of batched builds: parallel planning, tile shapes, per-XCD work
// queues, the on-device autotuner and HIP graph capture.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <numeric>
#include <thread>

#include "tn_batch.h"

namespace tn {
// Launch shape of a batch: slice halvings, threads per workgroup, LDS bytes
// a workgroup may take (a smaller budget fits more workgroups on a compute
// unit and sends the widest networks to global-memory tiles) and the slice
// width of global-memory tiles, in words.
struct BatchShape {
    int policy = 0;
    uint32_t threads = 1024;
    uint32_t lds = 163840;  // all of a compute unit's LDS on gfx950
    uint32_t gwidth = 8;
};
}  // namespace tn

struct tn_batch {
    int device = 0;
    int32_t B = 0;
    uint32_t flags = 0;
    std::vector<tn_plan_stats> stats;
    std::vector<tn::DevSchedule> views;
    std::vector<uint32_t> n, nwords;
    std::vector<int64_t> max_gat;
    void *dev_sched = nullptr;   // every schedule, one allocation
    // shapes
    std::vector<uint32_t> lw, mode;
    tn::BatchShape shape;
    uint32_t grid = 0;
    size_t dyn_lds = 0;
    int per_cu = 0;
    // device metadata
    void *dev_meta = nullptr;
    size_t meta_bytes = 0;
    tn::NetDesc *d_nets = nullptr;
    uint2 *d_tiles = nullptr;
    uint32_t *d_qptr = nullptr;
    uint32_t *d_counters = nullptr;
    uint64_t *d_gscratch = nullptr;
    std::vector<tn::NetDesc> h_nets;
    bool sat = true;  // saturation setting of the current shape
    // streamed chunk (tn::BatchStream): forced slice widths, slice state
    bool streamed = false;
    std::vector<uint32_t> force_lw;
    std::vector<uint32_t *> persist;
    uint32_t resume = 0;
    unsigned int *done_count = nullptr;
    std::vector<uint2> h_tiles;
    uint32_t h_qptr[9] = {0};
    int64_t lds_tiles = 0;
    // graph of the current shape
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    bool tuned = false;
    std::vector<uint64_t *> last_C;
    std::vector<int64_t> last_ld;
};

namespace tn {

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

uint32_t pow2_ceil(uint32_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

uint32_t ilog2(uint32_t x) {
    uint32_t l = 0;
    while ((1u << (l + 1)) <= x) ++l;
    return l;
}

// dynamic LDS bytes left of a workgroup budget
size_t lds_budget(size_t limit) { return limit - batch_static_lds() - 256; }

// Widest power-of-two slice (<= 64 words) whose rows plus compound scratch
// (plus the saturation bitmap when `sat`) fit in LDS; 0 if none does.
uint32_t lds_fit_words(uint32_t n, int64_t max_gat, uint32_t nwords, bool sat, size_t limit) {
    if (lds_budget(limit) < (sat ? sat_bitmap_bytes(n) : 0)) return 0;
    const size_t budget = lds_budget(limit) - (sat ? sat_bitmap_bytes(n) : 0);
    uint32_t w = std::min<uint32_t>(64, pow2_ceil(nwords));
    for (; w >= 1; w >>= 1)
        if ((size_t)(n + (size_t)max_gat) * w * 8 <= budget) return w;
    return 0;
}

void free_meta(tn_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    if (b->dev_meta) (void)hipFree(b->dev_meta);
    b->dev_meta = nullptr;
    b->meta_bytes = 0;
}

// Chooses tile shapes for `policy` (0: widest slice that fits, k: k halvings
// for more, smaller tiles), builds the LPT-ordered per-XCD queues and
// uploads the descriptors.
tn_status apply_shape(tn_ctx *ctx, tn_batch *b, const BatchShape &shape) {
    hipError_t se = hipStreamSynchronize(ctx->stream);
    if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
    free_meta(b);
    b->shape = shape;
    const int policy = shape.policy;
    const uint32_t threads = shape.threads;
    b->sat = ctx->saturation;
    const int32_t B = b->B;
    b->lw.assign(B, 0);
    b->mode.assign(B, kTileLds);
    std::vector<uint32_t> sat_on(B, 0), sat_off(B, 0);
    size_t dyn = 0, gscr_words = 0;
    std::vector<size_t> gscr_off(B, 0);
    struct T {
        double cost;
        uint32_t net, slice;
    };
    std::vector<T> tiles;
    b->lds_tiles = 0;
    for (int32_t i = 0; i < B; ++i) {
        const uint32_t nw = b->nwords[i];
        const size_t bm = sat_bitmap_bytes(b->n[i]);
        // the bitmap must fit beside the LDS tile, or alone for a global tile
        sat_on[i] = b->sat && bm <= lds_budget(shape.lds);
        uint32_t w = lds_fit_words(b->n[i], b->max_gat[i], nw, sat_on[i], shape.lds);
        if (b->streamed && !b->force_lw.empty()) {
            // the chunk keeps the stream's slices: LDS if that width fits
            const uint32_t fw = 1u << b->force_lw[i];
            if (w < fw) b->mode[i] = kTileGlobal;
            w = fw;
        } else if (w == 0) {
            b->mode[i] = kTileGlobal;
            w = std::min<uint32_t>(shape.gwidth, pow2_ceil(nw));
        }
        if (b->mode[i] == kTileGlobal && b->max_gat[i] > 0) {
            gscr_off[i] = gscr_words;
            gscr_words += (size_t)b->max_gat[i] * scratch_stride(nw);
        }
        if (!b->streamed) w = std::max<uint32_t>(1, w >> policy);
        b->lw[i] = ilog2(w);
        const size_t tile = (b->mode[i] == kTileLds) ? (size_t)(b->n[i] + (size_t)b->max_gat[i]) * w * 8 : 0;
        sat_off[i] = (uint32_t)(tile / 8);
        dyn = std::max(dyn, tile + (sat_on[i] ? bm : 0));
        const uint32_t slices = (nw + w - 1) / w;
        const tn_plan_stats &st = b->stats[i];
        // modeled tile time: a per-level barrier cost plus per-word row work
        const double unit = (b->mode[i] == kTileLds) ? 1.0 : 6.0;
        const double cost = (double)st.levels * 600.0 +
                            unit * (double)(st.pairs * 2 + st.gather_sources) * w * 8.0 / 4.0 +
                            (double)b->n[i] * w;
        for (uint32_t s = 0; s < slices; ++s) tiles.push_back({cost, (uint32_t)i, s});
        if (b->mode[i] == kTileLds) b->lds_tiles += slices;
    }
    std::stable_sort(tiles.begin(), tiles.end(), [](const T &a, const T &c) { return a.cost > c.cost; });
    // LPT over the 8 XCD queues
    double load[8] = {0};
    std::vector<std::vector<uint2>> q(8);
    for (const T &t : tiles) {
        int best = 0;
        for (int x = 1; x < 8; ++x)
            if (load[x] < load[best]) best = x;
        load[best] += t.cost;
        q[best].push_back(make_uint2(t.net, t.slice));
    }
    b->h_tiles.clear();
    b->h_qptr[0] = 0;
    for (int x = 0; x < 8; ++x) {
        b->h_tiles.insert(b->h_tiles.end(), q[x].begin(), q[x].end());
        b->h_qptr[x + 1] = (uint32_t)b->h_tiles.size();
    }
    b->dyn_lds = dyn;
    int per_cu = 0;
    hipError_t e = batch_occupancy((int)threads, dyn, &per_cu);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    if (per_cu < 1) return fail(TN_E_UNSUPPORTED, "batch kernel does not fit on a compute unit");
    b->per_cu = per_cu;
    const size_t ntiles = b->h_tiles.size();
    b->grid = (uint32_t)std::max<size_t>(1, std::min<size_t>((size_t)ctx->num_cus * per_cu, ntiles));
    // metadata allocation: nets, tiles, qptr, counters, global scratch
    size_t off = 0;
    const size_t o_nets = off; off = align256(off + sizeof(NetDesc) * B);
    const size_t o_tiles = off; off = align256(off + sizeof(uint2) * std::max<size_t>(ntiles, 1));
    const size_t o_qptr = off; off = align256(off + sizeof(uint32_t) * 9);
    const size_t o_cnt = off; off = align256(off + sizeof(uint32_t) * 8);
    const size_t o_scr = off; off = align256(off + sizeof(uint64_t) * std::max<size_t>(gscr_words, 1));
    e = hipMalloc(&b->dev_meta, off);
    if (e != hipSuccess) {
        b->dev_meta = nullptr;
        return fail(TN_E_NOMEM, "batch metadata allocation failed");
    }
    b->meta_bytes = off;
    unsigned char *base = (unsigned char *)b->dev_meta;
    b->d_nets = (NetDesc *)(base + o_nets);
    b->d_tiles = (uint2 *)(base + o_tiles);
    b->d_qptr = (uint32_t *)(base + o_qptr);
    b->d_counters = (uint32_t *)(base + o_cnt);
    b->d_gscratch = (uint64_t *)(base + o_scr);
    b->h_nets.assign(B, NetDesc{});
    for (int32_t i = 0; i < B; ++i) {
        NetDesc &nd = b->h_nets[i];
        nd.s = b->views[i];
        nd.C = nullptr;
        nd.ld = b->nwords[i];
        nd.nwords = b->nwords[i];
        nd.lw = b->lw[i];
        nd.mode = b->mode[i];
        nd.gscratch = b->d_gscratch + gscr_off[i];
        nd.sat = sat_on[i];
        nd.sat_off = sat_off[i];
        nd.resume = b->streamed ? b->resume : 0u;
        nd.persist = (b->streamed && sat_on[i] && !b->persist.empty()) ? b->persist[i] : nullptr;
    }
    e = hipMemcpy(b->d_tiles, b->h_tiles.data(), sizeof(uint2) * ntiles, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_qptr, b->h_qptr, sizeof(uint32_t) * 9, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch metadata upload");
    b->last_C.clear();
    b->last_ld.clear();
    return TN_OK;
}

tn_status bind_outputs(tn_ctx *ctx, tn_batch *b, uint64_t *const *C, const int64_t *ld) {
    bool same = b->last_C.size() == (size_t)b->B;
    for (int32_t i = 0; same && i < b->B; ++i) same = b->last_C[i] == C[i] && b->last_ld[i] == ld[i];
    if (same) return TN_OK;
    // a queued launch may still read the descriptors
    hipError_t se = hipStreamSynchronize(ctx->stream);
    if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
    for (int32_t i = 0; i < b->B; ++i) {
        NetDesc &nd = b->h_nets[i];
        nd.C = C[i];
        nd.ld = ld[i];
        nd.pair = nd.lw >= 1 && (nd.mode == kTileLds ||
                                 (ld[i] % 2 == 0 && ((uintptr_t)C[i] & 15u) == 0));
    }
    hipError_t e = hipMemcpy(b->d_nets, b->h_nets.data(), sizeof(NetDesc) * b->B,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");
    b->last_C.assign(C, C + b->B);
    b->last_ld.assign(ld, ld + b->B);
    return TN_OK;
}

hipError_t launch_direct(tn_batch *b, hipStream_t st) {
    return launch_batch(b->d_nets, b->d_tiles, b->d_qptr, b->d_counters, b->grid, b->shape.threads,
                        b->dyn_lds, b->done_count, st);
}

tn_status capture_graph(tn_batch *b) {
    if (b->exec) return TN_OK;
    hipError_t e;
    if (!b->cap_stream) {
        e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "capture stream");
    }
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = launch_direct(b, b->cap_stream);
    e = hipStreamEndCapture(b->cap_stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "batch launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->exec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return TN_OK;
}

// Times every candidate shape on the device and keeps the fastest.
tn_status autotune(tn_ctx *ctx, tn_batch *b, uint64_t *const *C, const int64_t *ld) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(TN_E_HIP, "event creation failed");
    float best_ms = 1e30f;
    bool found = false;
    BatchShape best;
    tn_status st = TN_OK;
    auto trial = [&](const BatchShape &c) -> bool {
        st = apply_shape(ctx, b, c);
        if (st == TN_E_UNSUPPORTED) {
            st = TN_OK;
            return true;
        }
        if (st != TN_OK) return false;
        st = bind_outputs(ctx, b, C, ld);
        if (st != TN_OK) return false;
        hipError_t e = hipEventRecord(e0, ctx->stream);
        if (e == hipSuccess) e = launch_direct(b, ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = hip_fail(e, "autotune launch");
            return false;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
            found = true;
        }
        return true;
    };
    // stage 1: LDS budget per workgroup x threads, widest slices; stage 2:
    // slice halvings and global tile width around the winner
    bool ok = true;
    for (uint32_t lds : {163840u, 81920u, 40960u, 20480u, 10240u})
        for (uint32_t th : {256u, 512u, 1024u})
            if (ok) ok = trial(BatchShape{0, th, lds, 8});
    if (ok && found) {
        const BatchShape s1 = best;
        for (int p = 0; p <= 2; ++p)
            for (uint32_t gw : {8u, 16u, 32u})
                if (ok && (p != 0 || gw != 8)) ok = trial(BatchShape{p, s1.threads, s1.lds, gw});
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok) return st;
    if (!found) return fail(TN_E_UNSUPPORTED, "no batch shape fits on a compute unit");
    st = apply_shape(ctx, b, best);
    if (st != TN_OK) return st;
    b->tuned = true;
    return TN_OK;
}

}  // namespace

// Plans B networks on host threads and uploads their schedules.
tn_status plan_batch(int32_t B, const uint32_t *n, const int64_t *m, const uint32_t *const *src,
                     const uint32_t *const *dst, const int64_t *const *t, uint32_t flags,
                     std::vector<HostSchedule> &hs, std::string &err,
                     const uint32_t *const *maps, uint32_t n_src, unsigned threads, int forms) {
    if (B <= 0) {
        err = "B must be > 0";
        return TN_E_ARG;
    }
    if (!n || !m || !src || !dst || !t) {
        err = "null batch array";
        return TN_E_ARG;
    }
    hs.assign(B, HostSchedule());
    std::vector<tn_status> sts(B, TN_OK);
    std::vector<std::string> errs(B);
    std::atomic<int32_t> next{0};
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned nth = std::min<unsigned>(threads ? threads : hw, (unsigned)B);
    auto worker = [&]() {
        for (;;) {
            const int32_t i = next.fetch_add(1);
            if (i >= B) return;
            sts[i] = plan_events(n[i], m[i], src[i], dst[i], t[i], flags, hs[i], errs[i],
                                 maps ? maps[i] : nullptr, n_src, forms);
        }
    };
    std::vector<std::thread> pool;
    for (unsigned k = 1; k < nth; ++k) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
    for (int32_t i = 0; i < B; ++i)
        if (sts[i] != TN_OK) {
            err = "network " + std::to_string(i) + ": " + errs[i];
            return sts[i];
        }
    return TN_OK;
}

tn_status batch_create(tn_ctx *ctx, int32_t B, const uint32_t *n, const int64_t *m,
                       const uint32_t *const *src, const uint32_t *const *dst,
                       const int64_t *const *t, uint32_t flags, tn_batch **out,
                       const uint32_t *const *maps, uint32_t n_src, const BatchStream *stream) {
    if (!ctx || !out) return fail(TN_E_ARG, "ctx or out is NULL");
    *out = nullptr;
    std::vector<HostSchedule> hs;
    std::string err;
    tn_status st = plan_batch(B, n, m, src, dst, t, flags, hs, err, maps, n_src, 0, kFormGather);
    if (st != TN_OK) return fail(st, err);
    return batch_from_plans(ctx, B, n, flags, hs, out, stream);
}

tn_status batch_from_plans(tn_ctx *ctx, int32_t B, const uint32_t *n, uint32_t flags,
                           std::vector<HostSchedule> &hs, tn_batch **out,
                           const BatchStream *stream) {
    if (!ctx || !out) return fail(TN_E_ARG, "ctx or out is NULL");
    *out = nullptr;
    if (B <= 0 || (int32_t)hs.size() != B) return fail(TN_E_ARG, "one schedule per network");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    tn_batch *b = new (std::nothrow) tn_batch();
    if (!b) return fail(TN_E_NOMEM, "batch allocation failed");
    b->device = ctx->device;
    b->B = B;
    b->flags = flags;
    std::vector<size_t> offs(B);
    size_t total = 0;
    for (int32_t i = 0; i < B; ++i) {
        offs[i] = total;
        total += align256(schedule_device_bytes(hs[i]));
    }
    hipError_t e = hipMalloc(&b->dev_sched, total);
    if (e != hipSuccess) {
        delete b;
        return fail(TN_E_NOMEM, "batch schedule allocation failed");
    }
    // the schedules go up array by array through the context's pinned ring
    // (SDMA copies on its stream, overlapped with the host copies into the
    // next slots); the alignment gaps between arrays are cleared first
    std::vector<SchedPiece> pieces;
    b->stats.resize(B);
    e = hipMemsetAsync(b->dev_sched, 0, total, ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(b->dev_sched);
        delete b;
        return hip_fail(e, "batch schedule clear");
    }
    for (int32_t i = 0; i < B; ++i) {
        schedule_pieces(hs[i], pieces);
        tn_status us = TN_OK;
        for (const SchedPiece &pc : pieces) {
            us = ring_upload(ctx, (unsigned char *)b->dev_sched + offs[i] + pc.off, pc.src, pc.bytes);
            if (us != TN_OK) break;
        }
        if (us != TN_OK) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(b->dev_sched);
            delete b;
            return us;
        }
        b->views.push_back(schedule_view(hs[i], (unsigned char *)b->dev_sched + offs[i]));
        fill_stats(hs[i], b->stats[i]);
        b->n.push_back(n[i]);
        b->nwords.push_back((n[i] + 63) / 64);
        b->max_gat.push_back(hs[i].max_level_gathers);
        hs[i] = HostSchedule();  // release host memory early
    }
    if (stream) {
        b->streamed = true;
        b->tuned = true;  // a chunk must run exactly once: no autotuning
        b->resume = stream->resume;
        b->done_count = stream->done_count;
        if (stream->lw) b->force_lw.assign(stream->lw, stream->lw + B);
        if (stream->persist) b->persist.assign(stream->persist, stream->persist + B);
    }
    tn_status st = apply_shape(ctx, b, BatchShape{});
    if (st != TN_OK) {
        free_meta(b);
        (void)hipFree(b->dev_sched);
        delete b;
        return st;
    }
    *out = b;
    return TN_OK;
}

tn_status batch_execute(tn_ctx *ctx, tn_batch *b, uint64_t *const *C, const int64_t *ld) {
    if (!ctx || !b) return fail(TN_E_ARG, "ctx or batch is NULL");
    if (!C || !ld) return fail(TN_E_ARG, "C or ld is NULL");
    if (b->device != ctx->device) return fail(TN_E_ARG, "batch lives on another device");
    for (int32_t i = 0; i < b->B; ++i) {
        if (!C[i]) return fail(TN_E_ARG, "C[" + std::to_string(i) + "] is NULL");
        if (ld[i] < (int64_t)b->nwords[i])
            return fail(TN_E_ARG, "ld[" + std::to_string(i) + "] < ceil(n/64)");
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    tn_status st;
    if (!b->tuned) {
        st = autotune(ctx, b, C, ld);
        if (st != TN_OK) return st;
    } else if (b->sat != ctx->saturation) {
        // the context's saturation setting changed: rebuild the shape
        st = apply_shape(ctx, b, b->shape);
        if (st != TN_OK) return st;
    }
    st = bind_outputs(ctx, b, C, ld);
    if (st != TN_OK) return st;
    hipError_t e;
    if (b->streamed) {
        ProfScope ps(ctx, TN_K_BATCH);
        e = launch_direct(b, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "batch launch");
        return TN_OK;
    }
    st = capture_graph(b);
    if (st != TN_OK) return st;
    {
        ProfScope ps(ctx, TN_K_BATCH);
        e = hipGraphLaunch(b->exec, ctx->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return TN_OK;
}

void batch_slice_log2(const tn_batch *b, std::vector<uint32_t> &lw) { lw = b->lw; }

void batch_set_persist(tn_batch *b, uint32_t *const *persist, unsigned int *done_count) {
    b->persist.assign(persist, persist + b->B);
    b->done_count = done_count;
    for (int32_t i = 0; i < b->B; ++i)
        b->h_nets[i].persist = b->h_nets[i].sat ? persist[i] : nullptr;
    b->last_C.clear();  // the next execution uploads the descriptors
}

void batch_destroy(tn_batch *b) {
    if (!b) return;
    DeviceGuard g(b->device);
    (void)hipDeviceSynchronize();
    free_meta(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->dev_sched) (void)hipFree(b->dev_sched);
    delete b;
}

}  // namespace tn

extern "C" {

tn_status tn_batch_create(tn_ctx *ctx, int32_t B, const uint32_t *n, const int64_t *m,
                          const uint32_t *const *src, const uint32_t *const *dst,
                          const int64_t *const *t, uint32_t flags, tn_batch **out) {
    return tn::batch_create(ctx, B, n, m, src, dst, t, flags, out);
}

tn_status tn_batch_execute(tn_ctx *ctx, tn_batch *batch, uint64_t *const *C, const int64_t *ld) {
    return tn::batch_execute(ctx, batch, C, ld);
}

tn_status tn_batch_get_stats(const tn_batch *b, tn_plan_stats *stats, int64_t *tiles,
                             int64_t *lds_tiles) {
    if (!b) return tn::fail(TN_E_ARG, "batch is NULL");
    if (stats)
        for (int32_t i = 0; i < b->B; ++i) stats[i] = b->stats[i];
    if (tiles) *tiles = (int64_t)b->h_tiles.size();
    if (lds_tiles) *lds_tiles = b->lds_tiles;
    return TN_OK;
}

tn_status tn_batch_get_shape(const tn_batch *batch, int64_t *shape) {
    if (!batch || !shape) return tn::fail(TN_E_ARG, "batch or shape is NULL");
    shape[0] = batch->shape.threads;
    shape[1] = (int64_t)batch->dyn_lds;
    shape[2] = batch->per_cu;
    shape[3] = batch->grid;
    shape[4] = batch->shape.policy;
    shape[5] = batch->shape.gwidth;
    return TN_OK;
}

void tn_batch_destroy(tn_batch *batch) { tn::batch_destroy(batch); }

tn_status tn_build_component_matrix_batched(tn_ctx *ctx, int32_t B, const uint32_t *n,
                                            const int64_t *m, const uint32_t *const *src,
                                            const uint32_t *const *dst, const int64_t *const *t,
                                            uint32_t flags, uint64_t *const *C, const int64_t *ld) {
    if (!C || !ld) return tn::fail(TN_E_ARG, "C or ld is NULL");
    for (int32_t i = 0; i < B; ++i)
        if (n && ld[i] < (int64_t)((n[i] + 63) / 64)) return tn::fail(TN_E_ARG, "ld < ceil(n/64)");
    tn_batch *b = nullptr;
    tn_status st = tn::batch_create(ctx, B, n, m, src, dst, t, flags, &b);
    if (st != TN_OK) return st;
    st = tn::batch_execute(ctx, b, C, ld);
    if (st == TN_OK) {
        tn::DeviceGuard g(ctx->device);
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = tn::hip_fail(e, "hipStreamSynchronize");
    }
    tn::batch_destroy(b);
    return st;
}

}  // extern "C"

namespace tn {

tn_status ring_upload(tn_ctx *ctx, void *dst, const void *src, size_t bytes) {
    constexpr size_t kSlot = (size_t)32 << 20;
    hipError_t e;
    if (!ctx->ring_buf[0]) {
        for (int i = 0; i < tn_ctx::kRingSlots; ++i) {
            e = hipHostMalloc(&ctx->ring_buf[i], kSlot, 0);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ring_ev[i], hipEventDisableTiming);
            if (e != hipSuccess) {
                ring_free(ctx);
                return fail(TN_E_NOMEM, "pinned upload ring allocation failed");
            }
        }
    }
    const unsigned char *p = (const unsigned char *)src;
    unsigned char *d = (unsigned char *)dst;
    while (bytes > 0) {
        const int k = ctx->ring_next;
        if (ctx->ring_busy[k]) {
            e = hipEventSynchronize(ctx->ring_ev[k]);
            if (e != hipSuccess) return hip_fail(e, "upload ring wait");
            ctx->ring_busy[k] = false;
        }
        const size_t c = std::min(bytes, kSlot);
        std::memcpy(ctx->ring_buf[k], p, c);
        e = hipMemcpyAsync(d, ctx->ring_buf[k], c, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(ctx->ring_ev[k], ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "upload ring copy");
        ctx->ring_busy[k] = true;
        ctx->ring_next = (k + 1) % tn_ctx::kRingSlots;
        p += c;
        d += c;
        bytes -= c;
    }
    return TN_OK;
}

// Frees the ring (the caller has waited for the context's stream).
void ring_free(tn_ctx *ctx) {
    for (int i = 0; i < tn_ctx::kRingSlots; ++i) {
        if (ctx->ring_ev[i]) (void)hipEventDestroy(ctx->ring_ev[i]);
        if (ctx->ring_buf[i]) (void)hipHostFree(ctx->ring_buf[i]);
        ctx->ring_ev[i] = nullptr;
        ctx->ring_buf[i] = nullptr;
        ctx->ring_busy[i] = false;
    }
    ctx->ring_next = 0;
}

}  // namespace tn
