// C ABI of network hashing (Sec. 4.1) and fusion (Sec. 4.2).
#include <algorithm>
#include <chrono>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "tn_batch.h"
#include "tn_hash.h"
#include "tn_wave.h"

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
    if (flags & TN_FORWARD) return fail(TN_E_ARG, "hashing takes no TN_FORWARD");
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
    // the host planner needs the bucket map of every hash: into the
    // context's pinned staging (one DMA, no page faults on a fresh array)
    st = ensure_host_staging(ctx, sizeof(uint32_t) * H * n);
    if (st != TN_OK) return st;
    const uint32_t *hb = (const uint32_t *)ctx->host_staging;
    e = hipMemcpyAsync(ctx->host_staging, bucket, sizeof(uint32_t) * H * n, hipMemcpyDeviceToHost,
                       ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "bucket download");
    std::vector<uint32_t> ns(H, K);
    std::vector<int64_t> ms(H, m);
    std::vector<const uint32_t *> ss(H, src), ds(H, dst), maps(H);
    std::vector<const int64_t *> ts(H, t);
    for (uint32_t j = 0; j < H; ++j) maps[j] = hb + (size_t)j * n;
    return batch_create(ctx, (int32_t)H, ns.data(), ms.data(), ss.data(), ds.data(), ts.data(),
                        flags, proxies, maps.data(), n);
}

}  // extern "C"

namespace tn {
namespace {
// Proxies of at most this many super-nodes run on one wavefront per column
// (timed on ER networks with Poisson events, K = 2100 to 3900: 1.4x to 2.2x
// faster than batched tiles; proxies that fill up within the first chunk
// lose the tiles' early stop there, a fraction of a millisecond).
constexpr uint32_t kWaveProxyK = 4096;

// Host image of one chunk of small proxies: the H op schedules at 256-byte
// aligned offsets off[j], then room for the H WaveNet records at off[H].
// Images are packed by the planner threads and recycled from chunk to
// chunk.  A long stream keeps them in pinned memory, so that an upload is
// one DMA; with few chunks the pinning would cost more than it saves.
struct WaveImage {
    unsigned char *pin = nullptr;
    size_t cap = 0;
    size_t bytes = 0;
    bool pinned = false;
    bool flat = false;  // the flat schedule format (k_rowor_wave_flat)
    std::vector<size_t> off;
    WaveImage() = default;
    WaveImage(const WaveImage &) = delete;
    WaveImage &operator=(const WaveImage &) = delete;
    WaveImage(WaveImage &&o) noexcept { swap(o); }
    WaveImage &operator=(WaveImage &&o) noexcept {
        swap(o);
        return *this;
    }
    ~WaveImage() { release(); }
    void swap(WaveImage &o) noexcept {
        std::swap(pin, o.pin);
        std::swap(cap, o.cap);
        std::swap(bytes, o.bytes);
        std::swap(pinned, o.pinned);
        std::swap(flat, o.flat);
        off.swap(o.off);
    }
    void release() {
        if (pin && pinned) (void)hipHostFree(pin);
        else delete[] pin;
        pin = nullptr;
        cap = 0;
    }
};

// Short levels (at most 80 ops on average) take the flat format: each op's
// rows as LDS byte offsets of a column of K real rows then the scratch rows,
// and a level-end bit, so that the kernel needs no level starts.
tn_status wave_image_pack(const std::vector<HostSchedule> &hs, uint32_t K, WaveImage &w,
                          bool pinned) {
    const uint32_t H = (uint32_t)hs.size();
    int64_t ops = 0, lv = 0;
    for (uint32_t j = 0; j < H; ++j) {
        ops += (int64_t)hs[j].ops.size() / 4;
        lv += hs[j].Lops;
    }
    w.flat = !rowor_wave_wide(ops, lv);
    w.off.assign(H + 1, 0);
    for (uint32_t j = 0; j < H; ++j) {
        const size_t bytes = w.flat ? flat_ops_bytes(hs[j]) : ops_device_bytes(hs[j]);
        w.off[j + 1] = w.off[j] + ((bytes + 255) & ~(size_t)255);
    }
    w.bytes = w.off[H] + sizeof(WaveNet) * H;
    if (w.bytes > w.cap || w.pinned != pinned) {
        const size_t cap = std::max(w.bytes, w.cap + w.cap / 2);
        w.release();
        w.pinned = pinned;
        if (pinned) {
            if (hipHostMalloc((void **)&w.pin, cap, 0) != hipSuccess) {
                w.pin = nullptr;
                return TN_E_NOMEM;
            }
        } else {
            w.pin = new (std::nothrow) unsigned char[cap];
            if (!w.pin) return TN_E_NOMEM;
        }
        w.cap = cap;
    }
    for (uint32_t j = 0; j < H; ++j) {
        const HostSchedule &s = hs[j];
        unsigned char *b = w.pin + w.off[j];
        if (!w.flat) {
            std::memcpy(b, s.lvl_op.data(), 4 * s.lvl_op.size());
            if (!s.ops.empty())
                std::memcpy(b + ((4 * s.lvl_op.size() + 255) & ~(size_t)255), s.ops.data(),
                            4 * s.ops.size());
            continue;
        }
        flat_ops_pack(s, K, reinterpret_cast<uint32_t *>(b));
    }
    return TN_OK;
}

// Device side of the upload: one buffer, grown as needed, kept across chunks.
struct WaveBuf {
    void *dev = nullptr;
    size_t cap = 0;
    ~WaveBuf() {
        if (dev) (void)hipFree(dev);
    }
};

// One chunk of small proxies: uploads the packed image, runs the H op
// schedules on one wavefront per word column of each proxy (slice state per
// column in state, col_words per proxy), reads the done count into
// *done_host and waits.
tn_status run_wave_chunk(tn_ctx *ctx, const std::vector<HostSchedule> &hs, WaveImage &img,
                         uint32_t K, const std::vector<uint64_t *> &Cs, int64_t ldK,
                         uint32_t *state, size_t col_words, unsigned int *done_dev,
                         unsigned int *done_host, int64_t &levels, WaveBuf &buf) {
    const uint32_t H = (uint32_t)hs.size();
    uint32_t max_scr = 0;
    int64_t ops = 0, lv = 0;
    for (uint32_t j = 0; j < H; ++j) {
        max_scr = std::max(max_scr, hs[j].scratch_rows);
        lv += hs[j].Lops;
        ops += (int64_t)hs[j].ops.size() / 4;
    }
    levels += lv;
    hipError_t e = hipSuccess;
    if (img.bytes > buf.cap) {
        // the previous chunk's copy and launch are complete (it was waited for)
        const size_t cap = std::max(img.bytes, buf.cap + buf.cap / 2);
        if (buf.dev) (void)hipFree(buf.dev);
        buf.dev = nullptr;
        buf.cap = 0;
        e = hipMalloc(&buf.dev, cap);
        if (e != hipSuccess) {
            buf.dev = nullptr;
            return fail(TN_E_NOMEM, "proxy schedule allocation failed");
        }
        buf.cap = cap;
    }
    unsigned char *dev = (unsigned char *)buf.dev;
    for (uint32_t j = 0; j < H; ++j) {
        WaveNet net;
        if (img.flat) {
            net.s = DevOps{hs[j].Lops, (uint32_t)(hs[j].ops.size() / 4), nullptr,
                           reinterpret_cast<const uint4 *>(dev + img.off[j])};
        } else {
            net.s = ops_view(hs[j], dev + img.off[j]);
        }
        net.C = Cs[j];
        net.ld = ldK;
        net.persist = ctx->saturation ? state + (size_t)j * col_words : nullptr;
        std::memcpy(img.pin + img.off[H] + sizeof(WaveNet) * j, &net, sizeof(WaveNet));
    }
    e = hipMemcpyAsync(dev, img.pin, img.bytes, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        ProfScope ps(ctx, TN_K_BATCH);
        if (img.flat)
            e = launch_rowor_wave_flat((const WaveNet *)(dev + img.off[H]), H, K, max_scr,
                                       ctx->saturation, done_dev, nullptr, ctx->stream);
        else
            e = launch_rowor_wave_multi((const WaveNet *)(dev + img.off[H]), H, K, max_scr,
                                        rowor_wave_wide(ops, lv), nullptr, ctx->saturation,
                                        done_dev, ctx->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(done_host, done_dev, sizeof(unsigned int), hipMemcpyDeviceToHost,
                           ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "proxy chunk");
    return TN_OK;
}
}  // namespace
}  // namespace tn

extern "C" {

// Streamed build of the H proxies (Sec. 4.3: the hashed networks are
// independent and built in parallel; Sec. 3.4: each is a reverse-time
// stream).  The event list is cut into chunks of whole time steps from its
// end; for each chunk the H mapped sub-streams are planned on host threads
// and applied in one batched launch that resumes from the proxies in HBM.
// Every tile carries its saturation state from chunk to chunk, and the
// build stops once every tile of every proxy is all ones.
tn_status tn_hash_build_proxies(tn_ctx *ctx, uint32_t n, int64_t m, const uint32_t *src,
                                const uint32_t *dst, const int64_t *t, uint32_t flags,
                                uint32_t H, uint32_t K, const uint64_t *coeffs, int32_t order,
                                uint32_t *bucket, int32_t *count, uint64_t *P, int64_t ldK,
                                int64_t chunk_events, tn_stream_stats *stats) {
    using namespace tn;
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return fail(TN_E_ARG, "ctx is NULL");
    if (n == 0 || H == 0 || K == 0 || order < 1) return fail(TN_E_ARG, "n, H, K and order must be > 0");
    if (K > 65536) return fail(TN_E_UNSUPPORTED, "K must be <= 65536");
    if (!coeffs || !bucket || !count || !P) return fail(TN_E_ARG, "null coefficient or output array");
    if (ldK < (int64_t)((K + 63) / 64)) return fail(TN_E_ARG, "ldK must be >= ceil(K/64)");
    if (chunk_events < 0) return fail(TN_E_ARG, "chunk_events must be >= 0");
    if (flags & ~(uint32_t)(TN_DIRECTED | TN_TIES_SEQUENTIAL))
        return fail(TN_E_ARG, "unknown flag bits (hashing takes TN_DIRECTED | TN_TIES_SEQUENTIAL)");
    for (size_t i = 0; i < (size_t)H * 3 * order; ++i)
        if (coeffs[i] >= kP61) return fail(TN_E_ARG, "hash coefficients must be < 2^61 - 1");
    if (m < 0 || (m > 0 && (!src || !dst || !t))) return fail(TN_E_ARG, "bad event arrays");
    if (m >= (int64_t)0xffffffffLL) return fail(TN_E_UNSUPPORTED, "m must be < 2^32 - 1");
    {
        std::string err;
        tn_status st = validate_events(n, m, src, dst, t, err);
        if (st != TN_OK) return fail(st, err);
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
    // the bucket maps into the context's pinned staging (one DMA, no page
    // faults on a fresh host array)
    st = ensure_host_staging(ctx, sizeof(uint32_t) * H * n);
    if (st != TN_OK) return st;
    const uint32_t *hb = (const uint32_t *)ctx->host_staging;
    e = hipMemcpyAsync(ctx->host_staging, bucket, sizeof(uint32_t) * H * n, hipMemcpyDeviceToHost,
                       ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "bucket download");
    int64_t first = 0;
    // proxies of K << n super-nodes saturate within few events: start small
    default_chunks(m, chunk_events, first, 16);
    std::vector<std::pair<int64_t, int64_t>> bounds;
    stream_chunks(m, t, chunk_events, first, flags & TN_TIES_SEQUENTIAL, false, bounds);
    if (bounds.empty()) bounds.emplace_back(0, 0);  // no events: identity proxies
    std::vector<uint32_t> ns(H, K);
    std::vector<const uint32_t *> maps(H);
    std::vector<uint64_t *> Cs(H);
    std::vector<int64_t> lds(H, ldK);
    for (uint32_t j = 0; j < H; ++j) {
        maps[j] = hb + (size_t)j * n;
        Cs[j] = P + (size_t)j * K * ldK;
    }
    // Small proxies (K <= kWaveProxyK) run as op schedules on one wavefront
    // per word column with the column in LDS (levels cost a few LDS round
    // trips there, against a barrier and schedule loads in the batched
    // kernel); larger ones as batched tiles.  One stream keeps one kind, as
    // the two keep different slice states, so the wavefront path is taken
    // only when every chunk's schedule fits it: the op planner never needs
    // more than max(default, K - 1) scratch rows for K nodes.
    const bool wave = K <= kWaveProxyK && rowor_wave_fits(K, std::max(kOpsScratchRows, K - 1));
    const uint32_t kw = (K + 63) / 64;
    const size_t wave_col = 2 * (size_t)((K + 31) / 32) + 2;  // slice state words per column
    std::vector<uint32_t> lw;
    std::vector<uint32_t *> pst(H, nullptr);
    uint32_t *state = nullptr;
    WaveBuf wbuf;
    unsigned int *done_host = nullptr;
    unsigned int *done_dev = nullptr;
    uint64_t tiles = 0;
    int64_t launched = 0, run_events = 0, levels = 0;
    bool all_done = false;
    e = hipHostMalloc((void **)&done_host, sizeof(unsigned int), 0);
    if (e != hipSuccess) return hip_fail(e, "pinned counter");
    *done_host = 0;
    // Chunk 0 is planned here on every host thread: its latency comes first,
    // and proxies of few super-nodes often saturate within it.  Only if they
    // do not, later chunks are planned by background threads, one proxy of
    // one chunk per task (so that few chunks still use every thread), ahead
    // of the launches by at most `window` chunks and about 2^26 mapped
    // events, so that host planning overlaps the device.
    const size_t nch = bounds.size();
    struct Planned {
        std::vector<HostSchedule> hs;
        WaveImage img;  // small proxies: the packed schedules
        tn_status st = TN_OK;
        std::string err;
        uint32_t left = 0;  // under mu: proxies of the chunk still being planned
        bool ready = false;
    };
    std::vector<WaveImage> spare;  // under mu: images of launched chunks
    std::vector<Planned> plans(nch);
    for (size_t c = 1; c < nch; ++c) {
        plans[c].hs.assign(H, HostSchedule());
        plans[c].left = H;
    }
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<size_t> next{H};  // background tasks: proxy j of chunk c is task c * H + j
    bool stop = false;    // under mu: no more chunks are wanted
    size_t consumed = 0;  // under mu: chunks launched
    bool pin_images = false;  // set below, before the first chunk is planned
    auto plan_chunk = [&](size_t c, unsigned threads) {
        const int64_t a = bounds[c].first, mc = bounds[c].second - bounds[c].first;
        std::vector<int64_t> ms(H, mc);
        std::vector<const uint32_t *> ss(H, src ? src + a : nullptr), ds(H, dst ? dst + a : nullptr);
        std::vector<const int64_t *> ts(H, t ? t + a : nullptr);
        std::vector<HostSchedule> hs;
        std::string err;
        const tn_status ps = plan_batch((int32_t)H, ns.data(), ms.data(), ss.data(), ds.data(),
                                        ts.data(), flags, hs, err, maps.data(), n, threads,
                                        wave ? kFormOps : kFormGather);
        WaveImage img;
        tn_status ws = TN_OK;
        if (wave && ps == TN_OK) {
            {
                std::lock_guard<std::mutex> lk(mu);
                if (!spare.empty()) {
                    img = std::move(spare.back());
                    spare.pop_back();
                }
            }
            // chunk 0 is uploaded once and its latency comes first: never pinned
            ws = wave_image_pack(hs, K, img, pin_images && c > 0);
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            plans[c].hs = std::move(hs);
            plans[c].img = std::move(img);
            plans[c].st = ps == TN_OK ? ws : ps;
            plans[c].err = ps == TN_OK && ws != TN_OK ? "schedule image allocation failed"
                                                      : std::move(err);
            plans[c].ready = true;
        }
        cv.notify_all();
    };
    // proxy j of chunk c >= 1, on a background thread; the last proxy of a
    // chunk to finish packs the chunk's image
    auto plan_one = [&](size_t c, uint32_t j) {
        const int64_t a = bounds[c].first, mc = bounds[c].second - bounds[c].first;
        HostSchedule h;
        std::string err;
        const tn_status ps = plan_events(K, mc, src ? src + a : nullptr, dst ? dst + a : nullptr,
                                         t ? t + a : nullptr, flags, h, err, maps[j], n,
                                         wave ? kFormOps : kFormGather);
        bool last;
        {
            std::lock_guard<std::mutex> lk(mu);
            plans[c].hs[j] = std::move(h);
            if (ps != TN_OK && plans[c].st == TN_OK) {
                plans[c].st = ps;
                plans[c].err = "network " + std::to_string(j) + ": " + err;
            }
            last = --plans[c].left == 0;
        }
        if (!last) return;
        // every other task of chunk c has finished: its schedules are ours
        WaveImage img;
        tn_status ws = TN_OK;
        if (wave && plans[c].st == TN_OK) {
            {
                std::lock_guard<std::mutex> lk(mu);
                if (!spare.empty()) {
                    img = std::move(spare.back());
                    spare.pop_back();
                }
            }
            ws = wave_image_pack(plans[c].hs, K, img, pin_images);
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            plans[c].img = std::move(img);
            if (ws != TN_OK && plans[c].st == TN_OK) {
                plans[c].st = ws;
                plans[c].err = "schedule image allocation failed";
            }
            plans[c].ready = true;
        }
        cv.notify_all();
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nth = std::min<size_t>(std::min<unsigned>(hw, 16u), (nch - 1) * H);
    const size_t window = std::max<size_t>(
        1, std::min<size_t>(nth, ((size_t)1 << 26) / std::max<size_t>(1, (size_t)H * chunk_events)));
    // at most window + 1 images are live at once: pin them when each is
    // reused a few times (chunk 0's never: pinning a fresh image costs
    // more than one pageable upload, at K = 4096, H = 16 about 7 ms)
    pin_images = nch >= 4 * (window + 1);
    auto worker = [&]() {
        (void)hipSetDevice(ctx->device);  // for the pinned image allocations
        for (;;) {
            const size_t task = next.fetch_add(1);
            const size_t c = task / H;
            if (c >= nch) return;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || c < consumed + window; });
                if (stop) return;
            }
            plan_one(c, (uint32_t)(task % H));
        }
    };
    plan_chunk(0, 0);
    std::vector<std::thread> pool;
    for (size_t c = 0; c < nch && st == TN_OK; ++c) {
        const int64_t mc = bounds[c].second - bounds[c].first;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return plans[c].ready; });
        }
        if (plans[c].st != TN_OK) {
            st = fail(plans[c].st, plans[c].err);
            break;
        }
        if (wave) {
            if (c == 0) {
                // per-column slice state of every proxy, the done counter;
                // the proxies start as the identity
                const size_t words = (size_t)H * kw * wave_col;
                e = hipMalloc((void **)&state, sizeof(uint32_t) * (words + 1));
                if (e != hipSuccess) {
                    state = nullptr;
                    st = fail(TN_E_NOMEM, "slice state allocation failed");
                    break;
                }
                done_dev = state + words;
                tiles = (uint64_t)H * kw;
                e = launch_fill_u32(state, words + 1, 0u, ctx->stream);
                for (uint32_t j = 0; j < H && e == hipSuccess; ++j)
                    e = launch_identity(Cs[j], K, ldK, nullptr, ctx->stream);
                if (e != hipSuccess) {
                    st = hip_fail(e, "proxy initialisation");
                    break;
                }
            }
            st = run_wave_chunk(ctx, plans[c].hs, plans[c].img, K, Cs, ldK, state, wave_col * kw,
                                done_dev, done_host, levels, wbuf);
            plans[c].hs.clear();
            if (st != TN_OK) break;
            ++launched;
            run_events += mc;
            {
                std::lock_guard<std::mutex> lk(mu);
                consumed = c + 1;
                spare.push_back(std::move(plans[c].img));
            }
            cv.notify_all();
            if (ctx->saturation && *done_host == tiles) {
                all_done = true;
                break;
            }
            if (c == 0)
                for (size_t k = 0; k < nth; ++k) pool.emplace_back(worker);
            continue;
        }
        BatchStream bs;
        bs.lw = c ? lw.data() : nullptr;
        bs.persist = c ? pst.data() : nullptr;
        bs.resume = c ? 1u : 0u;
        bs.done_count = done_dev;
        tn_batch *b = nullptr;
        st = batch_from_plans(ctx, (int32_t)H, ns.data(), flags, plans[c].hs, &b, &bs);
        plans[c].hs.clear();
        if (st != TN_OK) break;
        if (c == 0) {
            // slice state of every tile of every proxy, then the done counter
            batch_slice_log2(b, lw);
            std::vector<size_t> off(H + 1, 0);
            for (uint32_t j = 0; j < H; ++j) {
                off[j + 1] = off[j] + batch_persist_words(K, lw[j]);
                tiles += (((K + 63) / 64) + (1u << lw[j]) - 1) >> lw[j];
            }
            e = hipMalloc((void **)&state, sizeof(uint32_t) * (off[H] + 1));
            if (e != hipSuccess) {
                batch_destroy(b);
                st = fail(TN_E_NOMEM, "slice state allocation failed");
                break;
            }
            for (uint32_t j = 0; j < H; ++j) pst[j] = state + off[j];
            done_dev = state + off[H];
            e = launch_fill_u32(state, off[H] + 1, 0u, ctx->stream);
            if (e != hipSuccess) {
                batch_destroy(b);
                st = hip_fail(e, "slice state clear");
                break;
            }
            batch_set_persist(b, pst.data(), done_dev);
        }
        st = batch_execute(ctx, b, Cs.data(), lds.data());
        if (st == TN_OK) {
            e = hipMemcpyAsync(done_host, done_dev, sizeof(unsigned int), hipMemcpyDeviceToHost,
                               ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) st = hip_fail(e, "chunk completion");
        }
        std::vector<tn_plan_stats> bstats(H);
        (void)tn_batch_get_stats(b, bstats.data(), nullptr, nullptr);
        for (const auto &x : bstats) levels += x.levels;
        batch_destroy(b);
        if (st != TN_OK) break;
        ++launched;
        run_events += mc;
        {
            std::lock_guard<std::mutex> lk(mu);
            consumed = c + 1;
        }
        cv.notify_all();
        if (ctx->saturation && *done_host == tiles) {
            all_done = true;
            break;
        }
        if (c == 0)
            for (size_t k = 0; k < nth; ++k) pool.emplace_back(worker);
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv.notify_all();
    for (auto &th : pool) th.join();
    (void)hipStreamSynchronize(ctx->stream);
    if (state) (void)hipFree(state);
    (void)hipHostFree(done_host);
    if (stats) {
        stats->chunks = (int64_t)bounds.size();
        stats->chunks_run = launched;
        stats->events_run = run_events;
        stats->levels_run = levels;
        stats->saturated = all_done ? 1 : 0;
        stats->slice_words = wave ? 1 : (lw.empty() ? 0 : (int32_t)(1u << lw[0]));
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
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
    const size_t bs_bytes = align256((size_t)H * ((K + 63) / 64) * 4);
    const size_t lt_bytes = align256((size_t)qr * per_q);
    tn_status st =
        ensure_scratch(ctx, pt_bytes + rs_bytes + full_bytes + list_bytes + bs_bytes + lt_bytes);
    if (st != TN_OK) return st;
    unsigned char *base = (unsigned char *)ctx->scratch;
    uint64_t *PT = (uint64_t *)base;
    int32_t *rowsum = (int32_t *)(base + pt_bytes);
    uint8_t *full = base + pt_bytes + rs_bytes;
    uint32_t *list = (uint32_t *)(base + pt_bytes + rs_bytes + full_bytes);
    uint32_t *nlist_dev = list + n;
    int32_t *bsum = (int32_t *)(base + pt_bytes + rs_bytes + full_bytes + list_bytes);
    uint64_t *Lt = (uint64_t *)(base + pt_bytes + rs_bytes + full_bytes + list_bytes + bs_bytes);
    hipError_t e;
    uint32_t nlist = 0;
    {
        ProfScope ps(ctx, TN_K_AUX);
        // one pass over the proxies: full rows, and the lifted row sums
        e = launch_row_sums_full(H, K, ldK, P, count, bsum, lifted ? rowsum : nullptr, full,
                                 ctx->stream);
        if (e == hipSuccess && lifted)
            e = launch_lifted_sizes(n, H, K, bucket, rowsum, lifted, ctx->stream);
        if (e == hipSuccess)
            e = launch_split_full(n, H, K, bucket, full, est, list, nlist_dev, ctx->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(&nlist, nlist_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "recombine set-up kernels");
    // the transposed proxies feed the lifted tables only: none are needed
    // when every node's proxy rows are full in every hash (est = n)
    if (nlist > 0) {
        ProfScope ps(ctx, TN_K_AUX);
        e = launch_transpose_proxies(H, K, ldK, P, PT, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "proxy transpose launch");
    }
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
