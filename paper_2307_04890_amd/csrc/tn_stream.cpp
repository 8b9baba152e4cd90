// Streamed one-shot build of the exact component matrix.
//
// The reverse-time recurrence (Sec. 3.4) consumes the event list from its
// end.  The list is cut into chunks of whole time steps; chunk 0 holds the
// latest events.  Each chunk is planned on its own (levels start at 1; its
// compound scratch rows live inside it), so host threads plan several chunks
// at once, while the device runs the chunks strictly in order on the same
// matrix.  Rows only gain bits in reverse time, so once every row of a
// column slice is all ones nothing earlier in time can change that slice:
// the row-OR kernel carries each slice's saturation bits from one chunk to
// the next, a slice that is full returns at once, and the host stops
// planning and launching as soon as every slice is full.  A chunk launched
// after the last slice saturated only checks a flag, so the host polls the
// device's done counter without ever waiting for it.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>

#include "tn_internal.h"

namespace tn {

namespace {

struct Chunk {
    int64_t a = 0, b = 0;  // events [a, b)
    HostSchedule hs;
    std::vector<unsigned char> image;
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

}  // namespace

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

void stream_chunks(int64_t m, const int64_t *t, int64_t chunk, bool sequential,
                   std::vector<std::pair<int64_t, int64_t>> &out) {
    out.clear();
    for (int64_t b = m; b > 0;) {
        int64_t a = std::max<int64_t>(0, b - chunk);
        if (!sequential)
            while (a > 0 && t[a - 1] == t[a]) --a;
        out.emplace_back(a, b);
        b = a;
    }
}

tn_status build_streamed(tn_ctx *ctx, uint32_t n, int64_t m, const uint32_t *src,
                         const uint32_t *dst, const int64_t *t, uint32_t flags, uint64_t *C,
                         int64_t ld, int64_t chunk_events, tn_stream_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    if (!C) return fail(TN_E_ARG, "C is NULL");
    if (n == 0) return fail(TN_E_ARG, "n must be > 0");
    if (m < 0) return fail(TN_E_ARG, "m must be >= 0");
    if (m > 0 && (!src || !dst || !t)) return fail(TN_E_ARG, "null event array");
    if (flags & ~(uint32_t)(TN_DIRECTED | TN_TIES_SEQUENTIAL)) return fail(TN_E_ARG, "unknown flag bits");
    if (n > kNodeMask) return fail(TN_E_UNSUPPORTED, "n must be < 2^31");
    if (m >= (int64_t)0xffffffffLL) return fail(TN_E_UNSUPPORTED, "m must be < 2^32 - 1");
    if (chunk_events < 0) return fail(TN_E_ARG, "chunk_events must be >= 0");
    const int64_t nwords = (n + 63) / 64;
    if (ld < nwords) return fail(TN_E_ARG, "ld must be >= ceil(n/64)");
    {
        std::string err;
        tn_status st = validate_events(n, m, src, dst, t, err);
        if (st != TN_OK) return fail(st, err);
    }
    const bool seq = flags & TN_TIES_SEQUENTIAL;
    if (chunk_events == 0) chunk_events = std::max<int64_t>(1 << 18, (m + 63) / 64);
    // chunk boundaries from the end of the list, on time-step boundaries
    std::vector<std::pair<int64_t, int64_t>> bounds;
    stream_chunks(m, t, chunk_events, seq, bounds);
    std::vector<std::unique_ptr<Chunk>> chunks;
    for (const auto &ab : bounds) {
        auto c = std::make_unique<Chunk>();
        c->a = ab.first;
        c->b = ab.second;
        chunks.push_back(std::move(c));
    }
    const int64_t nch = (int64_t)chunks.size();

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(TN_E_HIP, "cannot select the context's device");
    const uint32_t sw = default_slice_words(n, ld);
    const uint32_t slices = rowor_workgroups(n, sw);
    hipError_t e;
    if (!ctx->traffic) {
        e = hipMalloc((void **)&ctx->traffic, 2 * sizeof(unsigned long long));
        if (e != hipSuccess) {
            ctx->traffic = nullptr;
            return fail(TN_E_NOMEM, "traffic counter allocation failed");
        }
    }
    // persisted slice state, then the done counter
    const size_t pwords = rowor_persist_words(n, sw);
    uint32_t *persist = nullptr;
    e = hipMalloc((void **)&persist, sizeof(uint32_t) * (pwords + 1));
    if (e != hipSuccess) return fail(TN_E_NOMEM, "slice state allocation failed");
    unsigned int *done_count = persist + pwords;
    Slot ring[kRing];
    auto release = [&]() {
        (void)hipStreamSynchronize(ctx->stream);
        for (Slot &s : ring) {
            if (s.dev) (void)hipFree(s.dev);
            if (s.pinned) (void)hipHostFree(s.pinned);
            if (s.done_host) (void)hipHostFree(s.done_host);
            if (s.ev) (void)hipEventDestroy(s.ev);
        }
        (void)hipFree(persist);
    };
    for (Slot &s : ring) {
        e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s.done_host, sizeof(unsigned int), 0);
        if (e != hipSuccess) {
            release();
            return hip_fail(e, "launch ring set-up");
        }
        *s.done_host = 0;
    }
    e = launch_fill_u32(persist, pwords + 1, 0u, ctx->stream);
    if (e == hipSuccess) {
        ProfScope ps(ctx, TN_K_IDENTITY);
        e = launch_identity(C, n, ld, ctx->traffic, ctx->stream);
    }
    if (e != hipSuccess) {
        release();
        return hip_fail(e, "identity kernel launch");
    }

    // planning workers: chunks in order, at most `window` ahead of the launches
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<int64_t> next{0};
    std::atomic<bool> stop{false};
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
                ch.st = plan_events(n, ch.b - ch.a, src + ch.a, dst + ch.a, t + ch.a, flags, ch.hs,
                                    ch.err, nullptr, 0, kFormOps);
                if (ch.st == TN_OK) ops_pack(ch.hs, ch.image);
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                ch.ready = true;
            }
            cv.notify_all();
        }
    };
    std::vector<std::thread> pool;
    for (int64_t k = 0; k < nth; ++k) pool.emplace_back(worker);
    auto finish = [&](tn_status st) {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        for (auto &th : pool) th.join();
        release();
        return st;
    };

    int64_t launched = 0, planned_events = 0, run_events = 0, levels = 0;
    bool all_done = false;
    tn_status st = TN_OK;
    for (int64_t c = 0; c < nch && !all_done; ++c) {
        Chunk &ch = *chunks[c];
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return ch.ready; });
        }
        if (ch.st != TN_OK) {
            st = fail(ch.st, ch.err);
            break;
        }
        // a completed earlier launch may already report every slice full
        for (int k = 0; k < kRing; ++k)
            if (ring[k].used && hipEventQuery(ring[k].ev) == hipSuccess &&
                *ring[k].done_host == slices)
                all_done = true;
        if (all_done) break;
        Slot &s = ring[c % kRing];
        if (s.used) {
            e = hipEventSynchronize(s.ev);
            if (e != hipSuccess) {
                st = hip_fail(e, "hipEventSynchronize");
                break;
            }
            if (*s.done_host == slices) {
                all_done = true;
                break;
            }
        }
        const size_t bytes = ch.image.size();
        if (bytes > s.dev_bytes) {
            if (s.dev) (void)hipFree(s.dev);
            s.dev = nullptr;
            s.dev_bytes = 0;
            e = hipMalloc(&s.dev, bytes);
            if (e != hipSuccess) {
                st = fail(TN_E_NOMEM, "chunk schedule allocation failed");
                break;
            }
            s.dev_bytes = bytes;
        }
        if (bytes > s.pinned_bytes) {
            if (s.pinned) (void)hipHostFree(s.pinned);
            s.pinned = nullptr;
            s.pinned_bytes = 0;
            e = hipHostMalloc(&s.pinned, bytes, 0);
            if (e != hipSuccess) {
                st = fail(TN_E_NOMEM, "chunk staging allocation failed");
                break;
            }
            s.pinned_bytes = bytes;
        }
        std::memcpy(s.pinned, ch.image.data(), bytes);
        const size_t need = sizeof(uint64_t) * ((size_t)slices * kRoworSinkWords +
                                                (size_t)ch.hs.scratch_rows * (size_t)nwords);
        st = ensure_scratch(ctx, need);
        if (st != TN_OK) break;
        e = hipMemcpyAsync(s.dev, s.pinned, bytes, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) {
            ProfScope ps(ctx, TN_K_ROWOR);
            e = launch_rowor_global(ops_view(ch.hs, s.dev), n, C, ld, sw, (uint64_t *)ctx->scratch,
                                    ch.hs.scratch_rows, ctx->traffic, ctx->saturation, persist,
                                    done_count, ctx->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(s.done_host, done_count, sizeof(unsigned int),
                               hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(s.ev, ctx->stream);
        if (e != hipSuccess) {
            st = hip_fail(e, "chunk launch");
            break;
        }
        s.used = true;
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
    for (int64_t c = 0; c < nch; ++c)
        if (chunks[c]->ready && chunks[c]->st == TN_OK) planned_events += chunks[c]->b - chunks[c]->a;
    if (st == TN_OK) {
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    if (st == TN_OK && !all_done)
        for (Slot &s : ring)
            if (s.used && *s.done_host == slices) all_done = true;
    if (stats) {
        stats->chunks = nch;
        stats->chunks_run = launched;
        stats->events_run = run_events;
        stats->levels_run = levels;
        stats->saturated = all_done ? 1 : 0;
        stats->slice_words = sw;
        stats->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    (void)planned_events;
    return finish(st);
}

}  // namespace tn

extern "C" {

tn_status tn_build_component_matrix_streamed(tn_ctx *ctx, uint32_t n, int64_t m,
                                             const uint32_t *src, const uint32_t *dst,
                                             const int64_t *t, uint32_t flags, uint64_t *C,
                                             int64_t ld, int64_t chunk_events,
                                             tn_stream_stats *stats) {
    return tn::build_streamed(ctx, n, m, src, dst, t, flags, C, ld, chunk_events, stats);
}

}  // extern "C"
