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
// level) fits the launch's LDS budget per workgroup is built entirely in
// LDS: identity, every level, then a single write-back of the slice.  Larger
// tiles run the same level loop on the matrix in global memory.  The host
// tunes the budget: levels are short, so a tile's time is mostly its levels'
// barrier and memory round trips, and a smaller budget lets several
// workgroups share a compute unit and hide each other's waits.
//
// Saturation (Sec. 3.4: rows only gain bits in reverse time).  A tile keeps
// one LDS bit per row meaning "this row is all ones in the slice": an item
// with a saturated operand reads nothing and gives a full result, a full
// result is not stored into a row already marked full, and every write
// refreshes the bit of the row it writes, so a set bit is always true.
// Once every row of the slice is full, nothing can change any more and the
// tile stops.
#include <hip/hip_runtime.h>

#include "tn_batch.h"
#include "tn_device.h"

namespace tn {

namespace {

constexpr uint32_t kWin = 64;  // levels of boundaries staged in LDS per window

// Rows of a tile; a lane holds LW consecutive words of a row (LW = 2:
// 16-byte accesses, which need every row to start on 16 bytes).
template <int LW>
struct LdsRows {
    using T = typename LaneT<LW>::T;
    uint64_t *M;
    uint32_t lw;  // log2(words per row)
    __device__ __forceinline__ T &at(uint32_t r, uint32_t lane) const {
        return *reinterpret_cast<T *>(&M[((size_t)r << lw) + LW * lane]);
    }
};

template <int LW>
struct GlobalRows {
    using T = typename LaneT<LW>::T;
    uint64_t *C;
    size_t ld;
    uint32_t word0;
    __device__ __forceinline__ T &at(uint32_t r, uint32_t lane) const {
        return *reinterpret_cast<T *>(&C[(size_t)r * ld + word0 + LW * lane]);
    }
};

// Saturation state of one tile.
template <int LW>
struct Sat {
    using T = typename LaneT<LW>::T;
    uint32_t *bits;  // LDS bitmap, bit r = row r is full in the slice
    int32_t *delta;  // per-level change of the full-row count, 3 slots
    T fullw;         // this lane's words of a full row slice (0 past the last word)
    T keep;          // clears a word past the last one (the matrix's padding)
    uint64_t gmask;  // ballot bits of this lane's group
    bool lead;       // first lane of its group
    __device__ __forceinline__ bool get(uint32_t r) const { return (bits[r >> 5] >> (r & 31u)) & 1u; }
    __device__ __forceinline__ void flip(uint32_t r, bool full, uint32_t l) const {
        if (full) atomicOr(&bits[r >> 5], 1u << (r & 31u));
        else atomicAnd(&bits[r >> 5], ~(1u << (r & 31u)));
        atomicAdd(&delta[l % 3], full ? 1 : -1);
    }
    // whether every lane of this lane's group has `mine` (all lanes of the
    // group are active together)
    __device__ __forceinline__ bool group_all(bool mine) const {
        return (__ballot(mine) & gmask) == gmask;
    }
};

// Runs every level of one network on one slice.  Rows and scratch are LDS or
// global views; `ok` masks lanes whose word is past the last word column
// (only needed for global views).  Lane groups of 2^lw lanes take the items
// of a level in turn; the next level's first items are prefetched into
// registers; level boundaries come from an LDS window refilled every kWin
// levels.
// Returns the number of full rows after the last level it ran (SAT).
template <int U, bool SAT, int LW, class Rows>
__device__ int32_t run_levels(const DevSchedule &s, const Rows rows, const Rows scr, uint32_t lw,
                              bool ok, uint32_t *winp, uint32_t *wing, const Sat<LW> &sat,
                              int32_t nfull) {
    using T = typename LaneT<LW>::T;
    const uint32_t tid = threadIdx.x;
    const uint32_t glw = lw - (LW == 2 ? 1u : 0u);  // log2 lanes per item
    const uint32_t lane = tid & ((1u << glw) - 1u);
    const uint32_t grp = tid >> glw;
    const uint32_t ngrp = blockDim.x >> glw;
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
    bool stopped = false;
    for (uint32_t l = 0; l < L; ++l) {
        if (SAT) {
            // every thread adds the same settled deltas: a uniform decision
            if (l > 0) nfull += sat.delta[(l - 1) % 3];
            if (nfull == (int32_t)s.n) {
                stopped = true;
                break;
            }
            if (tid == 0) sat.delta[(l + 1) % 3] = 0;
        }
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
            T a[U], b[U];
            bool fx[U], fy[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const bool v = it[k].x != 0xffffffffu;
                const uint32_t x = it[k].x, y = it[k].y & kNodeMask;
                fx[k] = SAT && v && sat.get(x);
                fy[k] = SAT && v && sat.get(y);
                a[k] = b[k] = T(0);
                if (v && ok && !fx[k] && !fy[k]) {
                    a[k] = rows.at(x, lane);
                    b[k] = rows.at(y, lane);
                }
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const bool v = it[k].x != 0xffffffffu, dir = it[k].y & kDirBit;
                const uint32_t x = it[k].x, y = it[k].y & kNodeMask;
                const T r = (fx[k] || fy[k]) ? sat.fullw : ((a[k] | b[k]) & sat.keep);
                bool full = false;
                if (SAT) full = sat.group_all(!v || !ok || lane_eq<LW>(r, sat.fullw));
                if (v && ok) {
                    if (!(full && fx[k])) rows.at(x, lane) = r;
                    if (!dir && !(full && fy[k])) rows.at(y, lane) = r;
                }
                if (SAT && v && sat.lead) {
                    if (full != fx[k]) sat.flip(x, full, l);
                    if (!dir && full != fy[k]) sat.flip(y, full, l);
                }
            }
        }
        if (g1 > g0) {
            // compound items: read every old row, then write
            for (uint32_t gi = g0 + grp; gi < g1; gi += ngrp) {
                T acc = T(0);
                const uint32_t s0 = s.gat_ptr[gi], s1 = s.gat_ptr[gi + 1];
                bool any_full = false;
                if (SAT)
                    for (uint32_t q = s0; q < s1 && !any_full; ++q) any_full = sat.get(s.gat_src[q]);
                if (ok) {
                    if (any_full) acc = sat.fullw;
                    else
                        for (uint32_t q = s0; q < s1; ++q) acc |= rows.at(s.gat_src[q], lane);
                    scr.at(gi - g0, lane) = acc & sat.keep;
                }
            }
            __syncthreads();
            for (uint32_t gi = g0 + grp; gi < g1; gi += ngrp) {
                const uint32_t tg = s.gat_tgt[gi];
                const T val = ok ? scr.at(gi - g0, lane) : T(0);
                if (!SAT) {
                    if (ok) rows.at(tg, lane) = val;
                    continue;
                }
                const bool ft = sat.get(tg);
                const bool full = sat.group_all(!ok || lane_eq<LW>(val, sat.fullw));
                if (ok && !(full && ft)) rows.at(tg, lane) = val;
                if (sat.lead && full != ft) sat.flip(tg, full, l);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < U; ++k) cur[k] = nxt[k];
        p0 = p1;
        p1 = p2;
        g0 = g1;
    }
    // the last level's delta settled at the loop's final barrier
    if (SAT && !stopped && L > 0) nfull += sat.delta[(L - 1) % 3];
    return nfull;
}

template <int U, bool SAT, int LW>
__device__ void run_tile(const NetDesc &nd, uint32_t slice, uint64_t *smem, uint32_t *winp,
                         uint32_t *wing, int32_t *fdelta, unsigned int *done_count) {
    using T = typename LaneT<LW>::T;
    const uint32_t tid = threadIdx.x;
    const uint32_t lw = nd.lw;
    const uint32_t w = 1u << lw;
    const uint32_t gw = w / LW;  // lanes per item
    const uint32_t n = nd.s.n;
    const uint32_t word0 = slice << lw;
    const size_t ld = (size_t)nd.ld;
    const uint32_t lane = tid & (gw - 1u);
    const uint32_t word = word0 + LW * lane;  // this lane's first word
    // saturation state; the bitmap is set up before the first barrier
    const uint32_t rwords = (n + 31) / 32;
    uint32_t *pst = (SAT && nd.persist) ? nd.persist + (size_t)slice * (rwords + 2) : nullptr;
    if (pst && pst[0]) return;  // this slice is all ones already (uniform)
    Sat<LW> sat;
    {
        // full value and padding mask of each of the lane's words
        const uint32_t tail = n & 63u;
        auto fw = [&](uint32_t wd) {
            return wd + 1 < nd.nwords ? ~0ull
                                      : (wd + 1 == nd.nwords ? (tail ? (1ull << tail) - 1ull : ~0ull)
                                                             : 0ull);
        };
        if constexpr (LW == 1) {
            sat.fullw = fw(word);
            sat.keep = ~0ull;
        } else {
            sat.fullw = u64x2{fw(word), fw(word + 1)};
            sat.keep = u64x2{~0ull, word + 1 < nd.nwords ? ~0ull : 0ull};
        }
    }
    int32_t nfull = 0;
    if (SAT) {
        sat.bits = (uint32_t *)(smem + nd.sat_off);
        sat.delta = fdelta;
        sat.gmask = (gw == 64 ? ~0ull : ((1ull << gw) - 1ull)) << ((tid & 63u) / gw * gw);
        sat.lead = lane == 0;
        // a slice with a single valid column starts with that row full
        const uint32_t c0 = word0 * 64u;
        const bool single = c0 + 1 == n;
        nfull = single ? 1 : 0;
        if (pst) {
            nfull = (int32_t)pst[1];
            if (single && !((pst[2 + (c0 >> 5)] >> (c0 & 31u)) & 1u)) ++nfull;
        }
        for (uint32_t i = tid; i < rwords; i += blockDim.x) {
            uint32_t v = pst ? pst[2 + i] : 0u;
            if (single && i == (c0 >> 5)) v |= 1u << (c0 & 31u);
            sat.bits[i] = v;
        }
        if (tid < 3) fdelta[tid] = 0;
    }
    if (nd.mode == kTileLds) {
        // identity on the slice in LDS, or the slice as earlier chunks left it
        const uint32_t total = n << lw;
        for (uint32_t i = tid; i < total; i += blockDim.x) {
            const uint32_t r = i >> lw, word = word0 + (i & (w - 1u));
            if (nd.resume)
                smem[i] = word < nd.nwords ? nd.C[(size_t)r * ld + word] : 0ull;
            else
                smem[i] = (word == (r >> 6)) ? (1ull << (r & 63u)) : 0ull;
        }
        __syncthreads();
        LdsRows<LW> rows{smem, lw};
        LdsRows<LW> scr{smem + total, lw};
        nfull = run_levels<U, SAT, LW>(nd.s, rows, scr, lw, true, winp, wing, sat, nfull);
        // write the slice back (the level loop ended with a barrier)
        for (uint32_t i = tid; i < total; i += blockDim.x) {
            const uint32_t r = i >> lw, word = word0 + (i & (w - 1u));
            if (word < nd.nwords) nd.C[(size_t)r * ld + word] = smem[i];
        }
    } else {
        const bool ok = word < nd.nwords;
        if (!nd.resume)
            for (size_t i = tid; i < ((size_t)n << lw); i += blockDim.x) {
                const uint32_t r = (uint32_t)(i >> lw), wd = word0 + (uint32_t)(i & (w - 1u));
                if (wd < nd.nwords)
                    nd.C[(size_t)r * ld + wd] = (wd == (r >> 6)) ? (1ull << (r & 63u)) : 0ull;
            }
        __syncthreads();
        GlobalRows<LW> rows{nd.C, ld, word0};
        // compound scratch rows lie an even number of words apart
        GlobalRows<LW> scr{nd.gscratch, (size_t)((nd.nwords + 1u) & ~1u), word0};
        nfull = run_levels<U, SAT, LW>(nd.s, rows, scr, lw, ok, winp, wing, sat, nfull);
    }
    if (pst) {
        for (uint32_t i = tid; i < rwords; i += blockDim.x) pst[2 + i] = sat.bits[i];
        if (tid == 0) {
            pst[1] = (uint32_t)nfull;
            if (nfull == (int32_t)n) {
                pst[0] = 1u;
                atomicAdd(done_count, 1u);
            }
        }
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
                   const uint32_t *__restrict__ qptr, uint32_t *__restrict__ counters,
                   unsigned int *__restrict__ done_count) {
    extern __shared__ uint64_t smem[];
    __shared__ uint32_t winp[2 * kWin], wing[2 * kWin];
    __shared__ uint32_t sh_tile;
    __shared__ int32_t fdelta[3];
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
            const NetDesc &nd = nets[tile.x];
            // two words per lane where the tile is at least two words wide
            // and its rows start on 16 bytes (NetDesc::pair)
            if (nd.sat) {
                if (nd.pair) run_tile<U, true, 2>(nd, tile.y, smem, winp, wing, fdelta, done_count);
                else run_tile<U, true, 1>(nd, tile.y, smem, winp, wing, fdelta, done_count);
            } else {
                if (nd.pair) run_tile<U, false, 2>(nd, tile.y, smem, winp, wing, fdelta, done_count);
                else run_tile<U, false, 1>(nd, tile.y, smem, winp, wing, fdelta, done_count);
            }
        }
    }
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

}  // namespace

size_t batch_static_lds() { return sizeof(uint32_t) * (4 * kWin + 1) + 3 * sizeof(int32_t); }

hipError_t batch_occupancy(int threads, size_t dyn_lds, int *blocks_per_cu) {
    hipError_t e = hipFuncSetAttribute((const void *)k_batch_persistent<4>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_persistent<4>,
                                                        threads, dyn_lds);
}

hipError_t launch_batch(const NetDesc *nets, const uint2 *tiles, const uint32_t *qptr,
                        uint32_t *counters, uint32_t grid, uint32_t threads, size_t dyn_lds,
                        unsigned int *done_count, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, counters, 8u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_persistent<4>, dim3(grid), dim3(threads), dyn_lds, st, nets, tiles,
                       qptr, counters, done_count);
    return hipGetLastError();
}

}  // namespace tn
