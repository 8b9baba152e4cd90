// Persistent multi-network row-OR kernel.
//
// A batch holds the level schedules of many networks (the H hashed proxies of
// Sec. 4.3, which are independent and can be built in parallel, or many
// unrelated temporal networks).  Every network's matrix is split into column
// slices of w words; a (network, slice) pair is a tile, and tiles never share
// a word, so they run in any order on any workgroup.  One launch of
// resident workgroups takes tiles from per-XCD work queues (largest first,
// then from the other XCDs' queues) until every queue is empty.
//
// A tile whose n x w slice (plus the scratch rows of its widest compound
// level) fits in LDS is built entirely in LDS: identity, every level, then a
// single write-back of the slice.  Larger tiles run the same level loop on
// the matrix in global memory.
#include <hip/hip_runtime.h>

#include "tn_batch.h"

namespace tn {

namespace {

constexpr uint32_t kWin = 64;  // levels of boundaries staged in LDS per window

struct LdsRows {
    uint64_t *M;
    uint32_t lw;  // log2(words per row)
    __device__ __forceinline__ uint64_t &at(uint32_t r, uint32_t lane) const {
        return M[((size_t)r << lw) + lane];
    }
};

struct GlobalRows {
    uint64_t *C;
    size_t ld;
    uint32_t word0;
    __device__ __forceinline__ uint64_t &at(uint32_t r, uint32_t lane) const {
        return C[(size_t)r * ld + word0 + lane];
    }
};

// Runs every level of one network on one slice.  Rows and scratch are LDS or
// global views; `ok` masks lanes whose word is past the last word column
// (only needed for global views).  Lane groups of 2^lw lanes take the items
// of a level in turn; the next level's first items are prefetched into
// registers; level boundaries come from an LDS window refilled every kWin
// levels.
template <int U, class Rows>
__device__ void run_levels(const DevSchedule &s, const Rows rows, const Rows scr, uint32_t lw,
                           bool ok, uint32_t *winp, uint32_t *wing) {
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & ((1u << lw) - 1u);
    const uint32_t grp = tid >> lw;
    const uint32_t ngrp = blockDim.x >> lw;
    const uint32_t chunk = ngrp * U;
    const uint32_t L = s.L;
    for (uint32_t i = tid; i < 2 * kWin; i += blockDim.x) {
        const uint32_t l = min(i, L);
        winp[i] = s.lvl_pair[l];
        wing[i] = s.lvl_gat[l];
    }
    __syncthreads();
    auto lp = [&](uint32_t l) { return winp[((l / kWin) & 1u) * kWin + l % kWin]; };
    auto lg = [&](uint32_t l) { return wing[((l / kWin) & 1u) * kWin + l % kWin]; };
    uint32_t p0 = lp(0), p1 = lp(1), g0 = lg(0);
    uint2 cur[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const uint32_t idx = p0 + grp + k * ngrp;
        cur[k] = idx < p1 ? s.pairs[idx] : make_uint2(0xffffffffu, 0u);
    }
    for (uint32_t l = 0; l < L; ++l) {
        if (l % kWin == 0 && l > 0) {
            const uint32_t nb = l / kWin + 1;
            for (uint32_t i = tid; i < kWin; i += blockDim.x) {
                const uint32_t ll = min(nb * kWin + i, L);
                winp[(nb & 1u) * kWin + i] = s.lvl_pair[ll];
                wing[(nb & 1u) * kWin + i] = s.lvl_gat[ll];
            }
        }
        const uint32_t p2 = lp(min(l + 2, L));
        const uint32_t g1 = lg(l + 1);
        uint2 nxt[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint32_t idx = p1 + grp + k * ngrp;
            nxt[k] = idx < p2 ? s.pairs[idx] : make_uint2(0xffffffffu, 0u);
        }
        for (uint32_t base = p0; base < p1; base += chunk) {
            uint2 it[U];
            if (base == p0) {
#pragma unroll
                for (int k = 0; k < U; ++k) it[k] = cur[k];
            } else {
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const uint32_t idx = base + grp + k * ngrp;
                    it[k] = idx < p1 ? s.pairs[idx] : make_uint2(0xffffffffu, 0u);
                }
            }
            uint64_t a[U], b[U];
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (it[k].x != 0xffffffffu && ok) {
                    a[k] = rows.at(it[k].x, lane);
                    b[k] = rows.at(it[k].y & kNodeMask, lane);
                }
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (it[k].x != 0xffffffffu && ok) {
                    const uint64_t r = a[k] | b[k];
                    rows.at(it[k].x, lane) = r;
                    if (!(it[k].y & kDirBit)) rows.at(it[k].y & kNodeMask, lane) = r;
                }
        }
        if (g1 > g0) {
            // compound items: read every old row, then write
            for (uint32_t gi = g0 + grp; gi < g1; gi += ngrp) {
                uint64_t acc = 0;
                const uint32_t s0 = s.gat_ptr[gi], s1 = s.gat_ptr[gi + 1];
                if (ok) {
                    for (uint32_t q = s0; q < s1; ++q) acc |= rows.at(s.gat_src[q], lane);
                    scr.at(gi - g0, lane) = acc;
                }
            }
            __syncthreads();
            for (uint32_t gi = g0 + grp; gi < g1; gi += ngrp)
                if (ok) rows.at(s.gat_tgt[gi], lane) = scr.at(gi - g0, lane);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < U; ++k) cur[k] = nxt[k];
        p0 = p1;
        p1 = p2;
        g0 = g1;
    }
}

template <int U>
__device__ void run_tile(const NetDesc &nd, uint32_t slice, uint64_t *smem, uint32_t *winp,
                         uint32_t *wing) {
    const uint32_t tid = threadIdx.x;
    const uint32_t lw = nd.lw;
    const uint32_t w = 1u << lw;
    const uint32_t n = nd.s.n;
    const uint32_t word0 = slice << lw;
    const size_t ld = (size_t)nd.ld;
    if (nd.mode == kTileLds) {
        // identity on the slice, in LDS
        const uint32_t total = n << lw;
        for (uint32_t i = tid; i < total; i += blockDim.x) {
            const uint32_t r = i >> lw, word = word0 + (i & (w - 1u));
            smem[i] = (word == (r >> 6)) ? (1ull << (r & 63u)) : 0ull;
        }
        __syncthreads();
        LdsRows rows{smem, lw};
        LdsRows scr{smem + total, lw};
        run_levels<U>(nd.s, rows, scr, lw, true, winp, wing);
        // write the slice back (the level loop ended with a barrier)
        for (uint32_t i = tid; i < total; i += blockDim.x) {
            const uint32_t r = i >> lw, word = word0 + (i & (w - 1u));
            if (word < nd.nwords) nd.C[(size_t)r * ld + word] = smem[i];
        }
    } else {
        const uint32_t lane = tid & (w - 1u);
        const bool ok = word0 + lane < nd.nwords;
        for (uint32_t r = tid >> lw; r < n; r += blockDim.x >> lw)
            if (ok) {
                const uint32_t word = word0 + lane;
                nd.C[(size_t)r * ld + word] = (word == (r >> 6)) ? (1ull << (r & 63u)) : 0ull;
            }
        __syncthreads();
        GlobalRows rows{nd.C, ld, word0};
        GlobalRows scr{nd.gscratch, (size_t)nd.nwords, word0};
        run_levels<U>(nd.s, rows, scr, lw, ok, winp, wing);
    }
    // padding words past the last word column are zero
    if (word0 + w >= nd.nwords && (size_t)nd.nwords < ld) {
        const uint32_t pad = (uint32_t)(ld - nd.nwords);
        for (size_t i = tid; i < (size_t)n * pad; i += blockDim.x)
            nd.C[(i / pad) * ld + nd.nwords + i % pad] = 0ull;
    }
    __syncthreads();  // LDS and the tile id are reused by the next tile
}

template <int U>
__global__ void __launch_bounds__(1024)
k_batch_persistent(const NetDesc *__restrict__ nets, const uint2 *__restrict__ tiles,
                   const uint32_t *__restrict__ qptr, uint32_t *__restrict__ counters) {
    extern __shared__ uint64_t smem[];
    __shared__ uint32_t winp[2 * kWin], wing[2 * kWin];
    __shared__ uint32_t sh_tile;
    const uint32_t x = blockIdx.x & 7u;
    for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t q = (x + k) & 7u;
        const uint32_t q0 = qptr[q], qn = qptr[q + 1] - q0;
        for (;;) {
            if (threadIdx.x == 0) sh_tile = atomicAdd(counters + q, 1u);
            __syncthreads();
            const uint32_t t = sh_tile;
            __syncthreads();
            if (t >= qn) break;
            const uint2 tile = tiles[q0 + t];
            run_tile<U>(nets[tile.x], tile.y, smem, winp, wing);
        }
    }
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

}  // namespace

size_t batch_static_lds() { return sizeof(uint32_t) * (4 * kWin + 1); }

hipError_t batch_occupancy(int threads, size_t dyn_lds, int *blocks_per_cu) {
    hipError_t e = hipFuncSetAttribute((const void *)k_batch_persistent<4>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_persistent<4>,
                                                        threads, dyn_lds);
}

hipError_t launch_batch(const NetDesc *nets, const uint2 *tiles, const uint32_t *qptr,
                        uint32_t *counters, uint32_t grid, uint32_t threads, size_t dyn_lds,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, counters, 8u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_persistent<4>, dim3(grid), dim3(threads), dyn_lds, st, nets, tiles,
                       qptr, counters);
    return hipGetLastError();
}

}  // namespace tn
