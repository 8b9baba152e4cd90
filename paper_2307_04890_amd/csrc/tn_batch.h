// Device descriptors and launchers of the persistent multi-network kernel.
#pragma once

#include "tn_internal.h"

namespace tn {

enum : uint32_t { kTileLds = 0, kTileGlobal = 1 };

// One network of a batch as the kernel sees it.
struct NetDesc {
    DevSchedule s;
    uint64_t *C;          // n x ld output matrix
    int64_t ld;
    uint32_t nwords;      // ceil(n / 64)
    uint32_t lw;          // log2 of the slice width in words
    uint32_t mode;        // kTileLds or kTileGlobal
    uint32_t sat;         // 1: track saturated rows in an LDS bitmap and stop early
    uint64_t *gscratch;   // global-mode compound scratch: max_gat x nwords words
    uint32_t sat_off;     // bitmap offset in the dynamic LDS, in uint64 words
    uint32_t resume;      // 1: start from the rows in C instead of the identity
    // per-slice state carried between launches over consecutive chunks of
    // one stream (nullable; sat only): {done, full-row count, ceil(n/32)
    // words of row bits} per slice, zero before the first chunk
    uint32_t *persist;
    // 1: lanes take two words of a row (16-byte accesses): slices of two or
    // more words whose rows start on 16 bytes (LDS tiles always, global
    // tiles with even ld and an aligned matrix)
    uint32_t pair;
};

// Bytes of the saturation bitmap of an n-node network (one bit per row).
inline size_t sat_bitmap_bytes(uint32_t n) { return (((size_t)n + 63) / 64) * 8; }

// Streamed use of a batch: every network is one chunk of a longer stream
// whose earlier chunks already ran on the same output matrices.
struct BatchStream {
    const uint32_t *lw = nullptr;      // forced log2 slice width per network (NULL: choose)
    uint32_t *const *persist = nullptr;  // per-network slice state (see NetDesc)
    uint32_t resume = 0;               // 1: the matrices hold the previous chunks
    unsigned int *done_count = nullptr;  // +1 per slice that becomes all full
};

// Plans B networks on host threads (node ids through maps[b] when given).
// With `stream`, the batch is launched directly at execution (no autotuning:
// re-running a chunk would apply its events twice).
tn_status batch_create(tn_ctx *ctx, int32_t B, const uint32_t *n, const int64_t *m,
                       const uint32_t *const *src, const uint32_t *const *dst,
                       const int64_t *const *t, uint32_t flags, tn_batch **out,
                       const uint32_t *const *maps = nullptr, uint32_t n_src = 0,
                       const BatchStream *stream = nullptr);
// The two halves of batch_create.  plan_batch plans the B networks on the
// host only (up to `threads` host threads, 0 = all; `forms` as for
// plan_events), so it may run on any thread; its error text goes to err.  batch_from_plans uploads them and
// sets the launch shape (device work: the calling thread must own the
// context's stream); it empties hs.
tn_status plan_batch(int32_t B, const uint32_t *n, const int64_t *m, const uint32_t *const *src,
                     const uint32_t *const *dst, const int64_t *const *t, uint32_t flags,
                     std::vector<HostSchedule> &hs, std::string &err,
                     const uint32_t *const *maps, uint32_t n_src, unsigned threads,
                     int forms = kFormGather);
tn_status batch_from_plans(tn_ctx *ctx, int32_t B, const uint32_t *n, uint32_t flags,
                           std::vector<HostSchedule> &hs, tn_batch **out,
                           const BatchStream *stream);
tn_status batch_execute(tn_ctx *ctx, tn_batch *b, uint64_t *const *C, const int64_t *ld);
void batch_destroy(tn_batch *b);
// log2 slice width each network of the batch uses
void batch_slice_log2(const tn_batch *b, std::vector<uint32_t> &lw);
// sets a streamed batch's slice state after creation (before its execution)
void batch_set_persist(tn_batch *b, uint32_t *const *persist, unsigned int *done_count);
// uint32 words of slice state of an n-node network with 2^lw-word slices
inline size_t batch_persist_words(uint32_t n, uint32_t lw) {
    const size_t nwords = ((size_t)n + 63) / 64, w = (size_t)1 << lw;
    return ((nwords + w - 1) / w) * (((size_t)n + 31) / 32 + 2);
}

size_t batch_static_lds();
hipError_t batch_occupancy(int threads, size_t dyn_lds, int *blocks_per_cu);
hipError_t launch_batch(const NetDesc *nets, const uint2 *tiles, const uint32_t *qptr,
                        uint32_t *counters, uint32_t grid, uint32_t threads, size_t dyn_lds,
                        unsigned int *done_count, hipStream_t st);

}  // namespace tn
