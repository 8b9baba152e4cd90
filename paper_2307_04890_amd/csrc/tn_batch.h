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
    uint32_t pad_;
};

// Bytes of the saturation bitmap of an n-node network (one bit per row).
inline size_t sat_bitmap_bytes(uint32_t n) { return (((size_t)n + 63) / 64) * 8; }

// Plans B networks on host threads (node ids through maps[b] when given).
tn_status batch_create(tn_ctx *ctx, int32_t B, const uint32_t *n, const int64_t *m,
                       const uint32_t *const *src, const uint32_t *const *dst,
                       const int64_t *const *t, uint32_t flags, tn_batch **out,
                       const uint32_t *const *maps = nullptr, uint32_t n_src = 0);

size_t batch_static_lds();
hipError_t batch_occupancy(int threads, size_t dyn_lds, int *blocks_per_cu);
hipError_t launch_batch(const NetDesc *nets, const uint2 *tiles, const uint32_t *qptr,
                        uint32_t *counters, uint32_t grid, uint32_t threads, size_t dyn_lds,
                        hipStream_t st);

}  // namespace tn
