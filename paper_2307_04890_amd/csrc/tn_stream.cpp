// Streamed builds of the component matrix: the one-shot call and online
// insertion.
//
// Algorithm 1 is a stream (Sec. 3.1): reverse time consumes the event list
// from its end (Sec. 3.4), forward time from its start.  A matrix that
// receives a stream keeps a device state (StreamState): the matrix itself,
// each column slice's saturation bits and full-row count, and a ring of
// launch buffers.  Events arrive in chunks of whole time steps.  Each chunk
// is planned on its own (levels start at 1; compound scratch rows live inside
// it), so host threads plan several chunks at once, while the device applies
// them strictly in stream order.  Rows only gain bits, so once every row of
// a column slice is all ones no further event can change that slice: the
// row-OR kernel carries each slice's saturation state from one launch to the
// next, a full slice returns at once, and the host stops planning and
// launching once every slice is full.  A chunk launched after the last slice
// saturated only checks a flag, so the host polls the device's done counter
// without ever waiting for it.
//
// The one-shot build is one state fed the whole list.  Online insertion
// (Sec. 3.5: new events and new nodes join a live matrix) keeps the state
// between calls; a node enters with its first event, its identity row being
// in place from the start.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>

#include "tn_internal.h"
#include "tn_wave.h"

namespace tn {

namespace {

struct Chunk {
    int64_t a = 0, b = 0;  // events [a, b)
    HostSchedule hs;
    std::vector<unsigned char> image;
    bool flat = false;  // the flat form, then room for one WaveNet (k_rowor_wave_flat)
    std::string err;
    tn_status st = TN_OK;
    bool ready = false;
};

// One device slot of the launch ring: a schedule buffer, its pinned staging
// copy, the done-counter snapshot taken after the launch that used it, and
// the event that marks that launch complete.
struct Slot {
    void *dev = nullptr;
    size_t dev_bytes = 0;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    unsigned int *done_host = nullptr;
    hipEvent_t ev = nullptr;
    bool used = false;
};

constexpr int kRing = 4;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Device state of one matrix that receives a stream chunk by chunk.
struct StreamState {
    uint32_t n = 0, flags = 0;
    uint64_t *C = nullptr;
    int64_t ld = 0;
    uint32_t sw = 0, slices = 0;
    uint32_t *persist = nullptr;  // per-slice state, then the done counter
    unsigned int *done_count = nullptr;
    Slot ring[kRing];
    int64_t launches = 0;  // launches so far (ring position)
    // zero phase: while every launch so far ran all its levels in it, the
    // persisted non-zero-row bits are exact and the next chunk may go on
    // with it, until the ops applied reach n
    bool zero_open = true;
    int64_t zero_ops = 0;
    bool all_done = false;
    bool has_time = false;
    int64_t edge_t = 0;  // latest (forward) or earliest (reverse) time applied
};

// Validates every event (ids < n, non-decreasing t) on several threads and
// reports the first offending event, as the single-threaded check would.
tn_status validate_events(uint32_t n, int64_t m, const uint32_t *src, const uint32_t *dst,
                          const int64_t *t, std::string &err) {
    if (m <= 0) return TN_OK;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t parts = std::max<int64_t>(1, std::min<int64_t>(hw, m / (1 << 20)));
    std::vector<int64_t> bad_id(parts, -1), bad_order(parts, -1);
    auto check = [&](int64_t p) {
        const int64_t e0 = m * p / parts, e1 = m * (p + 1) / parts;
        for (int64_t e = e0; e < e1; ++e) {
            if (src[e] >= n || dst[e] >= n) {
                bad_id[p] = e;
                break;
            }
            if (e > 0 && t[e] < t[e - 1]) {
                bad_order[p] = e;
                break;
            }
        }
    };
    std::vector<std::thread> th;
    for (int64_t p = 1; p < parts; ++p) th.emplace_back(check, p);
    check(0);
    for (auto &x : th) x.join();
    for (int64_t p = 0; p < parts; ++p) {
        if (bad_id[p] >= 0) {
            err = "event " + std::to_string(bad_id[p]) + " has a node id >= n";
            return TN_E_RANGE;
        }
        if (bad_order[p] >= 0) {
            err = "event " + std::to_string(bad_order[p]) + " is earlier than its predecessor";
            return TN_E_ORDER;
        }
    }
    return TN_OK;
}

void stream_chunks(int64_t m, const int64_t *t, int64_t chunk, int64_t first, bool sequential,
                   bool forward, std::vector<std::pair<int64_t, int64_t>> &out) {
    out.clear();
    int64_t size = first > 0 ? std::min(first, chunk) : chunk;
    auto grow = [&]() { size = std::min(chunk, 2 * size); };
    if (!forward) {
        for (int64_t b = m; b > 0;) {
            int64_t a = std::max<int64_t>(0, b - size);
            if (!sequential)
                while (a > 0 && t[a - 1] == t[a]) --a;
            out.emplace_back(a, b);
            b = a;
            grow();
        }
    } else {
        for (int64_t a = 0; a < m;) {
            int64_t b = std::min<int64_t>(m, a + size);
            if (!sequential)
                while (b < m && t[b] == t[b - 1]) ++b;
            out.emplace_back(a, b);
            a = b;
            grow();
        }
    }
}

void default_chunks(int64_t m, int64_t &chunk, int64_t &first, int shrink) {
    first = 0;
    if (chunk == 0) {
        chunk = std::max<int64_t>(1 << 18, (m + 63) / 64);
        first = std::max<int64_t>(1 << 14, chunk / shrink);
    }
}

namespace {

void state_release(tn_ctx *ctx, StreamState &s) {
    (void)hipStreamSynchronize(ctx->stream);
    for (Slot &r : s.ring) {
        if (r.dev) (void)hipFree(r.dev);
        if (r.pinned) (void)hipHostFree(r.pinned);
        if (r.done_host) (void)hipHostFree(r.done_host);
        if (r.ev) (void)hipEventDestroy(r.ev);
        r = Slot();
    }
    if (s.persist) (void)hipFree(s.persist);
    s.persist = nullptr;
}

// Allocates the state of an n-row matrix C and writes C <- I.
tn_status state_init(tn_ctx *ctx, StreamState &s, uint32_t n, uint32_t flags, uint64_t *C,
                     int64_t ld) {
    s.n = n;
    s.flags = flags;
    s.C = C;
    s.ld = ld;
    s.sw = default_slice_words(n, ld);
    s.slices = rowor_workgroups(n, s.sw);
    hipError_t e;
    if (!ctx->traffic) {
        e = hipMalloc((void **)&ctx->traffic, 2 * sizeof(unsigned long long));
        if (e != hipSuccess) {
            ctx->traffic = nullptr;
            return fail(TN_E_NOMEM, "traffic counter allocation failed");
        }
    }
    const size_t pwords = rowor_persist_words(n, s.sw);
    e = hipMalloc((void **)&s.persist, sizeof(uint32_t) * (pwords + 1));
    if (e != hipSuccess) {
        s.persist = nullptr;
        return fail(TN_E_NOMEM, "slice state allocation failed");
    }
    s.done_count = s.persist + pwords;
    for (Slot &r : s.ring) {
        e = hipEventCreateWithFlags(&r.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&r.done_host, sizeof(unsigned int), 0);
        if (e != hipSuccess) {
            state_release(ctx, s);
            return hip_fail(e, "launch ring set-up");
        }
        *r.done_host = 0;
    }
    e = launch_fill_u32(s.persist, pwords + 1, 0u, ctx->stream);
    if (e == hipSuccess) {
        ProfScope ps(ctx, TN_K_IDENTITY);
        e = launch_identity(C, n, ld, ctx->traffic, ctx->stream);
    }
    if (e != hipSuccess) {
        state_release(ctx, s);
        return hip_fail(e, "identity kernel launch");
    }
    return TN_OK;
}

// Applies events [0, m) (already validated) to the state in its direction:
// chunks planned on host threads, launched in stream order.  Returns once
// every chunk is launched (or the matrix is saturated); the launches may
// still run.
tn_status state_apply(tn_ctx *ctx, StreamState &s, int64_t m, const uint32_t *src,
                      const uint32_t *dst, const int64_t *t, int64_t chunk_events,
                      tn_stream_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    const bool seq = s.flags & TN_TIES_SEQUENTIAL;
    const bool forward = s.flags & TN_FORWARD;
    const int64_t nwords = (s.n + 63) / 64;
    int64_t first = 0;
    // the device time of the matrix stream dominates and planning runs ahead
    // of it, so its first chunk is only a quarter of the others
    default_chunks(m, chunk_events, first, 4);
    std::vector<std::pair<int64_t, int64_t>> bounds;
    stream_chunks(m, t, chunk_events, first, seq, forward, bounds);
    std::vector<std::unique_ptr<Chunk>> chunks;
    for (const auto &ab : bounds) {
        auto c = std::make_unique<Chunk>();
        c->a = ab.first;
        c->b = ab.second;
        chunks.push_back(std::move(c));
    }
    const int64_t nch = (int64_t)chunks.size();
    // Ring buffers are sized once for the largest chunk (its schedule image
    // as the planner reserves it: m + m/4 ops), so that the stream does not
    // reallocate as its chunks grow; a buffer that must grow all the same
    // is freed only after the stream, as hipFree would wait for the device.
    int64_t max_events = 0;
    for (const auto &c : chunks) max_events = std::max(max_events, c->b - c->a);
    const size_t reserve_ops = (size_t)max_events + (size_t)max_events / 4 + 4;
    const size_t image_guess = align256(4 * (reserve_ops + 1)) + align256(16 * reserve_ops);
    std::vector<void *> old_dev, old_pinned;
    // a completed launch may already report every slice full
    auto poll = [&]() {
        for (Slot &r : s.ring)
            if (r.used && hipEventQuery(r.ev) == hipSuccess && *r.done_host == s.slices)
                s.all_done = true;
    };
    poll();

    // planning workers: chunks in order, at most `window` ahead of the launches
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<int64_t> next{0};
    std::atomic<bool> stop{s.all_done};
    int64_t consumed = 0;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t nth = std::max<int64_t>(1, std::min<int64_t>(std::min<unsigned>(hw, 16u), nch));
    const int64_t window = 2 * nth;
    auto worker = [&]() {
        for (;;) {
            const int64_t c = next.fetch_add(1);
            if (c >= nch) return;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop.load() || c < consumed + window; });
            }
            Chunk &ch = *chunks[c];
            if (!stop.load()) {
                ch.st = plan_events(s.n, ch.b - ch.a, src + ch.a, dst + ch.a, t + ch.a, s.flags,
                                    ch.hs, ch.err, nullptr, 0, kFormOps);
                if (ch.st == TN_OK) {
                    // a chunk of short levels on the wavefront kernel takes
                    // the flat form (no level starts in the kernel's loop)
                    const int64_t nops = (int64_t)ch.hs.ops.size() / 4;
                    ch.flat = s.sw == 1 && rowor_wave_pays(s.n, ch.hs.scratch_rows, nops,
                                                           ch.hs.Lops) &&
                              !rowor_wave_wide(nops, ch.hs.Lops);
                    if (ch.flat) {
                        ch.image.assign(align256(flat_ops_bytes(ch.hs)) + sizeof(WaveNet), 0);
                        flat_ops_pack(ch.hs, s.n, reinterpret_cast<uint32_t *>(ch.image.data()));
                    } else {
                        ops_pack(ch.hs, ch.image);
                    }
                }
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                ch.ready = true;
            }
            cv.notify_all();
        }
    };
    std::vector<std::thread> pool;
    if (!s.all_done)
        for (int64_t k = 0; k < nth; ++k) pool.emplace_back(worker);

    int64_t launched = 0, run_events = 0, levels = 0;
    tn_status st = TN_OK;
    hipError_t e;
    for (int64_t c = 0; c < nch && !s.all_done; ++c) {
        Chunk &ch = *chunks[c];
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return ch.ready; });
        }
        if (ch.st != TN_OK) {
            st = fail(ch.st, ch.err);
            break;
        }
        poll();
        if (s.all_done) break;
        Slot &r = s.ring[s.launches % kRing];
        if (r.used) {
            e = hipEventSynchronize(r.ev);
            if (e != hipSuccess) {
                st = hip_fail(e, "hipEventSynchronize");
                break;
            }
            if (*r.done_host == s.slices) {
                s.all_done = true;
                break;
            }
        }
        const size_t bytes = ch.image.size();
        if (bytes > r.dev_bytes) {
            const size_t cap = std::max(std::max(bytes, image_guess), r.dev_bytes + r.dev_bytes / 2);
            if (r.dev) old_dev.push_back(r.dev);
            r.dev = nullptr;
            r.dev_bytes = 0;
            e = hipMalloc(&r.dev, cap);
            if (e != hipSuccess) {
                r.dev = nullptr;
                st = fail(TN_E_NOMEM, "chunk schedule allocation failed");
                break;
            }
            r.dev_bytes = cap;
        }
        if (bytes > r.pinned_bytes) {
            const size_t cap = std::max(std::max(bytes, image_guess), r.pinned_bytes + r.pinned_bytes / 2);
            if (r.pinned) old_pinned.push_back(r.pinned);
            r.pinned = nullptr;
            r.pinned_bytes = 0;
            e = hipHostMalloc(&r.pinned, cap, 0);
            if (e != hipSuccess) {
                r.pinned = nullptr;
                st = fail(TN_E_NOMEM, "chunk staging allocation failed");
                break;
            }
            r.pinned_bytes = cap;
        }
        std::memcpy(r.pinned, ch.image.data(), bytes);
        const size_t net_off = bytes - sizeof(WaveNet);  // flat: where the WaveNet goes
        if (ch.flat) {
            WaveNet net;
            net.s = DevOps{ch.hs.Lops, (uint32_t)(ch.hs.ops.size() / 4), nullptr,
                           reinterpret_cast<const uint4 *>(r.dev)};
            net.C = s.C;
            net.ld = s.ld;
            net.persist = ctx->saturation ? s.persist : nullptr;
            std::memcpy((unsigned char *)r.pinned + net_off, &net, sizeof(WaveNet));
        }
        const size_t need = sizeof(uint64_t) * ((size_t)s.slices * kRoworSinkWords +
                                                (size_t)ch.hs.scratch_rows *
                                                    (size_t)scratch_stride((uint32_t)nwords));
        st = ensure_scratch(ctx, need);
        if (st != TN_OK) break;
        e = hipMemcpyAsync(r.dev, r.pinned, bytes, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) {
            ProfScope ps(ctx, TN_K_ROWOR);
            uint32_t zl = 0;
            if (s.zero_open) {
                zl = zero_phase_levels(ch.hs, (int64_t)s.n - s.zero_ops);
                if (zl < ch.hs.Lops) s.zero_open = false;
                s.zero_ops += (int64_t)ch.hs.ops.size() / 4;
            }
            if (ch.flat)
                e = launch_rowor_wave_flat(
                    reinterpret_cast<const WaveNet *>((unsigned char *)r.dev + net_off), 1, s.n,
                    ch.hs.scratch_rows, ctx->saturation, s.done_count, ctx->traffic,
                    ctx->stream);
            else if (s.sw == 1 && rowor_wave_pays(s.n, ch.hs.scratch_rows,
                                                  (int64_t)ch.hs.ops.size() / 4, ch.hs.Lops))
                // a small network: one wavefront per word column; the slice
                // state goes on only when saturated slices may stop
                e = launch_rowor_wave(ops_view(ch.hs, r.dev), s.n, s.C, s.ld,
                                      ch.hs.scratch_rows, ctx->traffic, ctx->saturation,
                                      ctx->saturation ? s.persist : nullptr, s.done_count,
                                      ctx->stream);
            else
                e = launch_rowor_global(ops_view(ch.hs, r.dev), s.n, s.C, s.ld, s.sw,
                                        (uint64_t *)ctx->scratch, s.slices, ch.hs.scratch_rows,
                                        ctx->traffic, ctx->saturation, s.persist, s.done_count,
                                        zl, nullptr, ctx->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(r.done_host, s.done_count, sizeof(unsigned int),
                               hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(r.ev, ctx->stream);
        if (e != hipSuccess) {
            st = hip_fail(e, "chunk launch");
            break;
        }
        r.used = true;
        ++s.launches;
        ++launched;
        run_events += ch.b - ch.a;
        levels += ch.hs.Lops;
        // the host copy of this chunk is no longer needed
        ch.hs = HostSchedule();
        std::vector<unsigned char>().swap(ch.image);
        {
            std::lock_guard<std::mutex> lk(mu);
            ++consumed;
        }
        cv.notify_all();
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv.notify_all();
    for (auto &th : pool) th.join();
    if (!old_dev.empty() || !old_pinned.empty()) {
        // launches may still read the buffers that were replaced
        (void)hipStreamSynchronize(ctx->stream);
        for (void *p : old_dev) (void)hipFree(p);
        for (void *p : old_pinned) (void)hipHostFree(p);
    }
    if (stats) {
        stats->chunks = nch;
        stats->chunks_run = launched;
        stats->events_run = run_events;
        stats->levels_run = levels;
        stats->saturated = s.all_done ? 1 : 0;
        stats->slice_words = (int32_t)s.sw;
        stats->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

tn_status check_common(tn_ctx *ctx, uint32_t n, uint32_t flags, const uint64_t *C, int64_t ld) {
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    if (!C) return fail(TN_E_ARG, "C is NULL");
    if (n == 0) return fail(TN_E_ARG, "n must be > 0");
    if (flags & ~(uint32_t)(TN_DIRECTED | TN_TIES_SEQUENTIAL | TN_FORWARD))
        return fail(TN_E_ARG, "unknown flag bits");
    if (n > kNodeMask) return fail(TN_E_UNSUPPORTED, "n must be < 2^31");
    if (ld < (int64_t)((n + 63) / 64)) return fail(TN_E_ARG, "ld must be >= ceil(n/64)");
    return TN_OK;
}

tn_status check_events(int64_t m, const uint32_t *src, const uint32_t *dst, const int64_t *t,
                       int64_t chunk_events) {
    if (m < 0) return fail(TN_E_ARG, "m must be >= 0");
    if (m > 0 && (!src || !dst || !t)) return fail(TN_E_ARG, "null event array");
    if (m >= (int64_t)0xffffffffLL) return fail(TN_E_UNSUPPORTED, "m must be < 2^32 - 1");
    if (chunk_events < 0) return fail(TN_E_ARG, "chunk_events must be >= 0");
    return TN_OK;
}

}  // namespace

tn_status build_streamed(tn_ctx *ctx, uint32_t n, int64_t m, const uint32_t *src,
                         const uint32_t *dst, const int64_t *t, uint32_t flags, uint64_t *C,
                         int64_t ld, int64_t chunk_events, tn_stream_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    tn_status st = check_common(ctx, n, flags, C, ld);
    if (st == TN_OK) st = check_events(m, src, dst, t, chunk_events);
    if (st != TN_OK) return st;
    {
        std::string err;
        st = validate_events(n, m, src, dst, t, err);
        if (st != TN_OK) return fail(st, err);
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    StreamState s;
    st = state_init(ctx, s, n, flags, C, ld);
    if (st != TN_OK) return st;
    st = state_apply(ctx, s, m, src, dst, t, chunk_events, stats);
    if (st == TN_OK) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    if (st == TN_OK && stats) {
        // launches that completed after the last poll may have saturated it
        for (const Slot &r : s.ring)
            if (r.used && *r.done_host == s.slices) stats->saturated = 1;
        stats->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    state_release(ctx, s);
    return st;
}

}  // namespace tn

struct tn_online {
    tn_ctx *ctx = nullptr;
    tn::StreamState s;
};

extern "C" {

tn_status tn_build_component_matrix_streamed(tn_ctx *ctx, uint32_t n, int64_t m,
                                             const uint32_t *src, const uint32_t *dst,
                                             const int64_t *t, uint32_t flags, uint64_t *C,
                                             int64_t ld, int64_t chunk_events,
                                             tn_stream_stats *stats) {
    return tn::build_streamed(ctx, n, m, src, dst, t, flags, C, ld, chunk_events, stats);
}

tn_status tn_online_create(tn_ctx *ctx, uint32_t n, uint32_t flags, uint64_t *C, int64_t ld,
                           tn_online **out) {
    using namespace tn;
    if (!out) return fail(TN_E_ARG, "out is NULL");
    *out = nullptr;
    tn_status st = check_common(ctx, n, flags, C, ld);
    if (st != TN_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    tn_online *o = new (std::nothrow) tn_online();
    if (!o) return fail(TN_E_NOMEM, "online state allocation failed");
    o->ctx = ctx;
    st = state_init(ctx, o->s, n, flags, C, ld);
    if (st != TN_OK) {
        delete o;
        return st;
    }
    *out = o;
    return TN_OK;
}

tn_status tn_online_insert(tn_ctx *ctx, tn_online *o, int64_t m, const uint32_t *src,
                           const uint32_t *dst, const int64_t *t, int64_t chunk_events,
                           tn_stream_stats *stats) {
    using namespace tn;
    if (!ctx || !o) return fail(TN_E_ARG, "ctx or online state is NULL");
    if (o->ctx != ctx) return fail(TN_E_ARG, "online state belongs to another context");
    tn_status st = check_events(m, src, dst, t, chunk_events);
    if (st != TN_OK) return st;
    StreamState &s = o->s;
    {
        std::string err;
        st = validate_events(s.n, m, src, dst, t, err);
        if (st != TN_OK) return fail(st, err);
    }
    if (stats) *stats = tn_stream_stats{};
    if (m == 0) return TN_OK;
    // events of one time step must arrive in one call (they form one
    // snapshot), so a call continues strictly after what is applied
    const bool forward = s.flags & TN_FORWARD, seq = s.flags & TN_TIES_SEQUENTIAL;
    if (s.has_time) {
        const bool ok = forward ? (seq ? t[0] >= s.edge_t : t[0] > s.edge_t)
                                : (seq ? t[m - 1] <= s.edge_t : t[m - 1] < s.edge_t);
        if (!ok)
            return fail(TN_E_ORDER, forward ? "inserted events are not later than those applied"
                                            : "inserted events are not earlier than those applied");
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    st = state_apply(ctx, s, m, src, dst, t, chunk_events, stats);
    if (st == TN_OK) {
        s.has_time = true;
        s.edge_t = forward ? t[m - 1] : t[0];
    }
    return st;
}

void tn_online_destroy(tn_online *o) {
    if (!o) return;
    tn::DeviceGuard g(o->ctx->device);
    tn::state_release(o->ctx, o->s);
    delete o;
}

}  // extern "C"
