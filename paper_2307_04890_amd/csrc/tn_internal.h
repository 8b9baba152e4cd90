// Internal declarations shared by the host planner, the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tn.h"

namespace tn {

// Pair item encoding: {u, v | kDirBit}.  Undirected pair: both rows <- u | v.
// Directed pair (kDirBit set): row u <- u | v, row v unchanged.
constexpr uint32_t kDirBit = 0x80000000u;
constexpr uint32_t kNodeMask = 0x7fffffffu;

// Binary-op encoding {a, b, d1, d2}: r = row[a] | row[b]; row[d1] = r;
// row[d2] = r unless d2 == kNoRow.  A row id with kScratchBit set names a
// scratch row (compound items fold through them).  Levels hold at most
// kOpsLevelCap ops.
constexpr uint32_t kScratchBit = 0x80000000u;
constexpr uint32_t kNoRow = 0xffffffffu;
constexpr uint32_t kOpsLevelCap = 1024;
constexpr uint32_t kOpsScratchRows = 1024;
enum : int { kFormGather = 1, kFormOps = 2 };

// A single network's schedule on the host.  Items are sorted by level;
// level l owns pairs [lvl_pair[l], lvl_pair[l+1]) and gathers
// [lvl_gat[l], lvl_gat[l+1]).  Gather g writes row gat_tgt[g] with the OR of
// rows gat_src[gat_ptr[g] .. gat_ptr[g+1]) read before any gather of its
// level writes.
struct HostSchedule {
    uint32_t n = 0;
    int64_t m = 0;
    uint32_t flags = 0;
    uint32_t L = 0;
    std::vector<uint32_t> lvl_pair;  // L + 1
    std::vector<uint32_t> lvl_gat;   // L + 1
    std::vector<uint32_t> pairs;     // 2 * P (u, v | dir)
    std::vector<uint32_t> gat_tgt;   // G
    std::vector<uint32_t> gat_ptr;   // G + 1
    std::vector<uint32_t> gat_src;   // S
    int64_t compound_items = 0;
    int64_t directed_pairs = 0;
    // binary-op form (kFormOps): level l owns ops [lvl_op[l], lvl_op[l+1]),
    // 4 uint32 each
    uint32_t Lops = 0;
    uint32_t op_levels_unsplit = 0;
    uint32_t scratch_rows = 0;
    std::vector<uint32_t> lvl_op;  // Lops + 1
    std::vector<uint32_t> ops;     // 4 * nops
    int64_t op_pairs = 0, op_directed = 0, op_targets = 0, op_sources = 0, op_compound = 0;
    int64_t max_level_items = 0;
    int64_t max_level_gathers = 0;
    double host_seconds = 0.0;
};

// Forwarded op form, for the plain row-OR kernel that keeps each level's
// results in LDS for the next level (launch_rowor_fwd).  Levels hold at most
// kFwdLevelCap ops.  An operand with kFwdHot set is the result of op
// (operand & kFwdSlotMask) of the level just before, read from LDS; any
// other operand is a row id as in the op form (last written two or more
// levels before).  A destination with kFwdNoStore set is not stored: the
// next level overwrites that row (kNoRow carries the bit too).  Row and
// scratch ids stay below 2^30.  Levels hold at most `cap` ops (0 or more
// than kFwdLevelCap: kFwdLevelCap, what the kernels take; smaller caps are
// for tests of the splitting).  A level split into parts loses forwarding
// between them: an op moved to a later part no longer directly follows the
// writes of the level before.  Within a level, an op with one operand from
// memory has it second (y; the OR is symmetric), and ops with both operands
// from memory come first: the 16-word kernel holds x registers for the
// first ops only.
constexpr uint32_t kFwdLevelCap = 768;
constexpr uint32_t kFwdHot = 0x40000000u;
constexpr uint32_t kFwdNoStore = 0x40000000u;
constexpr uint32_t kFwdSlotMask = 0x3ffu;
void fwd_schedule(const std::vector<uint32_t> &lvl_op, const std::vector<uint32_t> &ops,
                  uint32_t n, uint32_t scratch_rows, uint32_t cap, std::vector<uint32_t> &flvl,
                  std::vector<uint32_t> &fops);

// Device view of one schedule (all pointers into one allocation).
struct DevSchedule {
    uint32_t n;
    uint32_t L;
    uint32_t max_gat;      // widest level, in gathers
    uint32_t pad_;
    const uint32_t *lvl_pair;
    const uint32_t *lvl_gat;
    const uint2 *pairs;
    const uint32_t *gat_tgt;
    const uint32_t *gat_ptr;
    const uint32_t *gat_src;
};

// Device view of a binary-op schedule: level l owns ops [lvl[l], lvl[l+1]).
struct DevOps {
    uint32_t L;
    uint32_t nops;
    const uint32_t *lvl;
    const uint4 *ops;
};

// Validates events and builds the schedule.  Returns TN_OK or an error code
// with `err` set.
// With `map`, event endpoints are ids < n_src sent through map[] to the n
// nodes of a hashed network.
// `forms` selects the gather form (pairs + gathers, for the batched kernel),
// the binary-op form (for the global kernel), or both.
tn_status plan_events(uint32_t n, int64_t m, const uint32_t *src,
                      const uint32_t *dst, const int64_t *t, uint32_t flags,
                      HostSchedule &out, std::string &err,
                      const uint32_t *map = nullptr, uint32_t n_src = 0,
                      int forms = kFormGather);

// Size in bytes of the device image of a schedule and its packing.
size_t schedule_device_bytes(const HostSchedule &s);
void schedule_pack(const HostSchedule &s, std::vector<unsigned char> &image);
DevSchedule schedule_view(const HostSchedule &s, const void *dev_base);
size_t ops_device_bytes(const HostSchedule &s);
void ops_pack(const HostSchedule &s, std::vector<unsigned char> &image);
DevOps ops_view(const HostSchedule &s, const void *dev_base);

// ---- error reporting and device scope (tn_abi.cpp) ---------------------
tn_status fail(tn_status code, const std::string &msg);
tn_status hip_fail(hipError_t e, const char *what);
tn_status not_built(const char *what);

// Makes a device current for the scope of an entry point.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace tn

struct tn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    // pinned host memory for device-to-host copies within one call (the
    // bucket maps of the hashed builds), kept for the next call
    void *host_staging = nullptr;
    size_t host_staging_bytes = 0;
    // row words loaded / stored by the last tn_plan_execute (device)
    unsigned long long *traffic = nullptr;
    // the slice state the last tn_plan_execute left in scratch (null: none)
    // and its slice width: a slice with its done word set is all ones in
    // every row of the matrix that execution wrote
    const uint32_t *state = nullptr;
    uint32_t state_sw = 0;
    // ring of pinned slots for host-to-device uploads (tn::ring_upload):
    // each slot's copy is an SDMA transfer on the context's stream, and its
    // event says when the slot may be refilled
    static constexpr int kRingSlots = 4;
    void *ring_buf[kRingSlots] = {};
    hipEvent_t ring_ev[kRingSlots] = {};
    bool ring_busy[kRingSlots] = {};
    int ring_next = 0;
    bool saturation = true;
    int num_cus = 0;
    // kernel timing (tn_profile_enable)
    bool profiling = false;
    struct Rec {
        int32_t id;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

struct tn_plan {
    int device = 0;
    void *dev = nullptr;
    size_t dev_bytes = 0;
    tn::DevOps view{};
    // the same ops in the flat form, for small networks whose levels are
    // short (one wavefront per word column; null otherwise)
    const uint32_t *flat = nullptr;
    uint32_t scratch_rows = 0;
    uint32_t zero_levels = 0;  // levels of the zero phase (tn::zero_phase_levels)
    // the op schedule on the host, and its forwarded form on the device,
    // made by the first execution of the plain recurrence (tn::fwd_schedule)
    std::vector<uint32_t> host_lvl_op, host_ops;
    mutable std::mutex fwd_mu;
    mutable void *fwd_dev = nullptr;
    mutable tn::DevOps fwd_view{};
    // ... and of op levels [zero_levels, mid_end) alone: the forwarding phase
    // of the saturating path (tn::kFwdPhaseOpsPerNode)
    uint32_t mid_end = 0;
    mutable void *mid_dev = nullptr;
    mutable tn::DevOps mid_view{};
    // TN_HLL plans: the time-step schedule (pairs and gathers by level) on
    // the device, its level boundaries on the host, instead of the ops
    bool hll = false;
    tn::DevSchedule gview{};
    std::vector<uint32_t> lvl_pair, lvl_gat;
    // ... and their level launches captured in a HIP graph, for the register
    // rows, scratch and row width they were captured with (replaced when one
    // changes; the mutex keeps concurrent calls on one plan apart)
    mutable std::mutex hll_mu;
    mutable std::vector<hipGraphExec_t> hll_execs;  // segments of tn::kHllSegmentLevels levels
    mutable const void *hll_M = nullptr, *hll_scr = nullptr;
    mutable uint32_t hll_nwords = 0;
    mutable bool hll_sat = false;
    tn_plan_stats stats{};
};

namespace tn {
// Brackets one kernel launch with events on the context's stream when
// profiling is on.
struct ProfScope {
    tn_ctx *c;
    size_t idx = (size_t)-1;
    ProfScope(tn_ctx *ctx, int32_t id) : c(ctx) {
        if (!c->profiling) return;
        hipEvent_t ev[2];
        for (int i = 0; i < 2; ++i) {
            if (!c->pool.empty()) {
                ev[i] = c->pool.back();
                c->pool.pop_back();
            } else if (hipEventCreate(&ev[i]) != hipSuccess) {
                for (int k = 0; k < i; ++k) c->pool.push_back(ev[k]);
                return;
            }
        }
        (void)hipEventRecord(ev[0], c->stream);
        c->recs.push_back({id, ev[0], ev[1]});
        idx = c->recs.size() - 1;
    }
    ~ProfScope() {
        if (idx != (size_t)-1) (void)hipEventRecord(c->recs[idx].b, c->stream);
    }
};

// Copies `bytes` from host memory to device memory through the context's
// ring of pinned slots (allocated on first use, freed by tn_destroy):
// asynchronous on the context's stream, and the source may be reused or
// freed as soon as the call returns.
tn_status ring_upload(tn_ctx *ctx, void *dst, const void *src, size_t bytes);
void ring_free(tn_ctx *ctx);
// The arrays of a schedule's device image (schedule_pack): offset in the
// image, host data, bytes.
struct SchedPiece {
    size_t off;
    const void *src;
    size_t bytes;
};
void schedule_pieces(const HostSchedule &s, std::vector<SchedPiece> &out);

// Grows the context scratch to at least `bytes`.
tn_status ensure_scratch(tn_ctx *ctx, size_t bytes);
// Grows the context's pinned host staging buffer to at least `bytes`
// (waits for the context's stream first; the buffer serves one call at a
// time, like the device scratch).
tn_status ensure_host_staging(tn_ctx *ctx, size_t bytes);
void fill_stats(const HostSchedule &hs, tn_plan_stats &s);

// ---- kernel launchers (tn_kernels.hip) ---------------------------------
// p[0 .. count) = v (a kernel, so it may be captured in a graph).
hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t v, hipStream_t st);
// traffic (nullable): two device counters the identity kernel zeroes.
hipError_t launch_identity(uint64_t *C, uint32_t n, int64_t ld, unsigned long long *traffic,
                           hipStream_t st);
// sink words per workgroup: one 16-byte slot per thread
constexpr size_t kRoworSinkWords = 2048;
// Scratch rows lie an even number of words apart, so that an access of two
// words at an even word stays on a 16-byte boundary.
inline uint32_t scratch_stride(uint32_t nwords) { return (nwords + 1u) & ~1u; }
// LDS bytes the saturation bitmap may take next to the op frames and work
// lists (gfx950: 160 KiB per workgroup).
constexpr size_t kRoworSatLds = 163840 - 40960;
// scratch: kRoworSinkWords words for each of sink_slots workgroups (at
// least rowor_workgroups(n, slice_words), else hipErrorInvalidValue), then
// scratch_rows rows of ceil(n/64) words, scratch_stride(ceil(n/64)) apart;
// launches that hand scratch rows over to each other pass the same
// sink_slots.  order (nullable): the slice each workgroup takes, in
// dispatch order (launch_slice_order), for the launch of the levels after
// zero_levels.
// The kernel adds the row words it loaded to traffic[0] and stored to
// traffic[1] (device counters, zeroed by the caller).  With saturation, and
// when a bit per row and scratch row fits kRoworSatLds, it skips the loads
// and stores that saturated rows make redundant; when two such bitmaps fit,
// also those that rows still all zero in a slice make redundant: with
// persist, the first zero_levels levels run as a launch of their own that
// tracks zero rows too (zero_phase_levels gives the number for a schedule
// that starts from the identity, 0 turns the phase off).  persist (nullable, only
// used with saturation): rowor_persist_words(n, slice_words) uint32 of
// per-slice state carried between launches over consecutive chunks of one
// stream, zero before the first; a slice that becomes all full sets its
// done word and adds 1 to *done_count.
uint32_t rowor_workgroups(uint32_t n, uint32_t slice_words);
hipError_t launch_rowor_global(const DevOps &s, uint32_t n, uint64_t *C, int64_t ld,
                               uint32_t slice_words, uint64_t *scratch, uint32_t sink_slots,
                               uint32_t scratch_rows, unsigned long long *traffic,
                               bool saturation, uint32_t *persist, unsigned int *done_count,
                               uint32_t zero_levels, const uint32_t *order, hipStream_t st);
// The plain recurrence (no saturation) on a forwarded op schedule
// (fwd_schedule), one workgroup per slice of slice_words <= 8 words as in
// launch_rowor_global, with the same scratch layout and traffic counters;
// each level's results stay in LDS for the next level.
bool rowor_fwd_supported(uint32_t n, uint32_t slice_words);
hipError_t launch_rowor_fwd(const DevOps &s, uint32_t n, uint64_t *C, int64_t ld,
                            uint32_t slice_words, uint64_t *scratch, uint32_t sink_slots,
                            uint32_t scratch_rows, unsigned long long *traffic, hipStream_t st);
// Rebuilds launch_rowor_global's per-slice state (persist, zeroed here
// first) from the matrix: the full-row bits and count of every slice, so
// that a saturating launch can resume after launches that kept no state
// (slice_words 1, 2, 4, 8 or 16, else hipErrorInvalidValue).
hipError_t launch_slice_full_state(const uint64_t *C, int64_t ld, uint32_t n,
                                   uint32_t slice_words, uint32_t *persist, hipStream_t st);
// The dispatch order of a saturating launch's slices (order: one uint32 per
// slice of slice_words words) from a slice state: fewest full real rows
// first, ties by slice index.
hipError_t launch_slice_order(const uint32_t *persist, uint32_t n, uint32_t slice_words,
                              uint32_t *order, hipStream_t st);
// The slice width of the saturating launch after the forwarding phase: a
// workgroup's busy level is bound by its own memory pipeline (the
// instructions and row segments it issues), so a slice still far from full
// takes time in proportion to its width, and the slowest slice sets the
// launch's time.  slice_words is halved while the slices stay within four
// per compute unit (one resident workgroup each; the slices with the most
// work go first and light ones fill the units that free up).  Row-OR at
// n = 10^5, m = 10^7 activity-driven, forwarding phase to 9 n: 2-word
// slices (782 workgroups) 15.1 ms, 4-word 15.5 ms; to 10 n: 2, 4 and 8 words
// 15.5, 15.8 and 15.9 ms.
uint32_t tail_slice_words(uint32_t n, uint32_t slice_words, int num_cus);
// The saturating path's middle phase: from the end of the zero phase until
// its ops reach kFwdPhaseOpsPerNode * n, the forwarding kernel (no skips,
// each level's results through LDS) runs instead of the saturating one;
// timed on the 10^5-node activity-driven workload, it is cheaper over that
// range and dearer after it, when most ops have a full operand (row-OR with
// the phase to 7, 8, 9, 10 and 11 n: 15.95, 15.30, 15.12, 15.46, 15.83 ms).
constexpr int64_t kFwdPhaseOpsPerNode = 9;
// Levels of the zero phase of a schedule: those before the level at which
// its ops reach `budget`.  Applied to the identity the budget is n (about
// one op per row), by when few row slices are still all zero; a streamed
// build spends it over its first chunks.
inline uint32_t zero_phase_levels(const HostSchedule &hs, int64_t budget) {
    uint32_t l = 0;
    while (l < hs.Lops && (int64_t)hs.lvl_op[l] < budget) ++l;
    return l;
}
// uint32 words of persisted state: per slice, done + count + ceil(n/32)
// full-row bits + ceil(n/32) non-zero-row bits
inline size_t rowor_persist_words(uint32_t n, uint32_t slice_words) {
    return (size_t)rowor_workgroups(n, slice_words) * (2 * (((size_t)n + 31) / 32) + 2);
}
// ids < n and non-decreasing t for every event, checked on several host
// threads; the message names the first offending event (tn_stream.cpp)
tn_status validate_events(uint32_t n, int64_t m, const uint32_t *src, const uint32_t *dst,
                          const int64_t *t, std::string &err);
// chunks of a time-ordered list in the order they are applied: taken from
// its end (reverse time) or, with forward, from its start; each of about
// `chunk` events and of whole time steps unless `sequential`.  With
// first > 0 the first chunk has about `first` events and each next one
// twice as many as the one before, up to `chunk` (tn_stream.cpp).
void stream_chunks(int64_t m, const int64_t *t, int64_t chunk, int64_t first, bool sequential,
                   bool forward, std::vector<std::pair<int64_t, int64_t>> &out);
// chunk == 0 (the default): chunk = max(2^18, m/64) events, and a first
// chunk of max(2^14, chunk/shrink) that doubles up to it, so that a stream
// that saturates early plans and runs little; an explicit chunk is kept
// fixed (first = 0)
void default_chunks(int64_t m, int64_t &chunk, int64_t &first, int shrink);
// The row-OR kernel with rows merged by byte-wise maximum (HyperLogLog
// registers below 128, nwords = 2, 4, 8, ... words per row of M, ld >=
// nwords); scratch as for launch_rowor_global with rowmax_workgroups sinks.
hipError_t launch_rowmax_global(const DevOps &s, uint32_t rows, uint32_t nwords, uint64_t *M,
                                int64_t ld, uint64_t *scratch, uint32_t scratch_rows,
                                unsigned long long *traffic, hipStream_t st);
uint32_t rowmax_workgroups(uint32_t nwords);
// HyperLogLog kernels (tn_hll.hip): every node's registers for its own hash,
// and the size estimates
hipError_t launch_hll_init(uint32_t n, uint32_t log2s, const uint64_t *node_hash, uint8_t *M,
                           hipStream_t st);
// The register stream of a TN_HLL plan, levels [l0, l1): one launch per
// level (pairs, and compound items' reads into scratch), then one writing
// the compound items' rows; scratch: s.max_gat rows of nwords words.  With
// Grow and left (saturation; both nullable): Grow is the register-wise
// maximum over every node's own registers and *left the rows not equal to
// it; a row that reaches Grow takes one off, and a level returns at once
// when *left is 0 (launch_hll_saturation_setup computes both, with gmax
// 2^log2s uint32 of scratch).
hipError_t launch_hll_levels(const DevSchedule &s, const uint32_t *lvl_pair,
                             const uint32_t *lvl_gat, uint32_t l0, uint32_t l1, uint32_t nwords,
                             uint64_t *M, uint64_t *scratch, const uint64_t *Grow,
                             unsigned int *left, hipStream_t st);
hipError_t launch_hll_saturation_setup(uint32_t n, uint32_t log2s, const uint64_t *node_hash,
                                       const uint8_t *M, unsigned int *gmax, uint64_t *Grow,
                                       unsigned int *left, hipStream_t st);
// Levels per captured graph of a TN_HLL plan; between graphs the host reads
// *left and stops once it is 0.
constexpr uint32_t kHllSegmentLevels = 256;
hipError_t launch_hll_estimate(uint32_t n, uint32_t log2s, const uint8_t *M, double *est,
                               hipStream_t st);
// streamed one-shot build (tn_stream.cpp)
tn_status build_streamed(tn_ctx *ctx, uint32_t n, int64_t m, const uint32_t *src,
                         const uint32_t *dst, const int64_t *t, uint32_t flags, uint64_t *C,
                         int64_t ld, int64_t chunk_events, tn_stream_stats *stats);
// whether the saturating kernel can run for n rows and this many scratch rows
inline bool rowor_saturates(uint32_t n, uint32_t scratch_rows) {
    const uint64_t sbits = (((uint64_t)n + 31) & ~31ull) + scratch_rows + 1;
    return ((sbits + 31) / 32) * 4 <= kRoworSatLds;
}
// Row and column popcounts of C; with a slice state (persist of slices of
// state_sw words, nullable) the words of slices left all ones are counted
// without a read.
hipError_t launch_out_sizes(const uint64_t *C, uint32_t n, int64_t ld, int32_t *out_sizes,
                            hipStream_t st, const uint32_t *persist = nullptr,
                            uint32_t state_sw = 0);
hipError_t launch_in_sizes(const uint64_t *C, uint32_t n, int64_t ld, int32_t *in_sizes,
                           hipStream_t st, const uint32_t *persist = nullptr,
                           uint32_t state_sw = 0);
uint32_t default_slice_words(uint32_t n, int64_t ld);

}  // namespace tn
