// gfx950 kernels of the row-OR stream of small networks: one wavefront per
// word column keeps the column of every row in LDS (Sec. 3.1 Algorithm 1 in
// reverse time, Sec. 3.4; each word column evolves on its own).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tn_device.h"
#include "tn_wave.h"

namespace tn {

namespace {

// Small networks: one wavefront per word column keeps that column of every
// row and scratch row in LDS and runs every level of the op schedule with
// no barrier.  The ops of a level touch disjoint rows, and one wavefront's
// LDS accesses complete in program order, so level l + 1 sees level l.
// The loop is software-pipelined so that a group of up to 64 ops of one
// level costs one LDS round trip.  Ops and level starts each live in an LDS
// ring of two windows; the window after those is loaded from HBM into
// registers one window ahead of use.  The next group's ops and the start
// of the level after next are read from LDS before the current group's row
// reads, so the level loop never waits on HBM or on a second LDS trip.
constexpr uint32_t kWaveWin = 512;
constexpr uint32_t kWaveRing = 2 * kWaveWin;
constexpr uint32_t kWavePre = kWaveWin / 64;  // entries per lane of a prefetched window

// A ring of two windows of T in LDS fed from src[0 .. count) (the last
// entry repeated past the end), with the window after them in registers.
template <typename T>
struct WaveRing {
    T *ring;
    const T *src;
    uint32_t count, nwin, next;  // windows below next are (or were) in the ring
    T pre[kWavePre];
    __device__ void fetch(uint32_t win, uint32_t lane) {
#pragma unroll
        for (uint32_t k = 0; k < kWavePre; ++k) pre[k] = src[min(win * kWaveWin + 64 * k + lane, count - 1)];
    }
    __device__ void store(uint32_t win, uint32_t lane) {
#pragma unroll
        for (uint32_t k = 0; k < kWavePre; ++k) ring[(win * kWaveWin + 64 * k + lane) % kWaveRing] = pre[k];
    }
    __device__ void init(T *r, const T *s, uint32_t c, uint32_t lane) {
        ring = r;
        src = s;
        count = c;
        nwin = (c + kWaveWin - 1) / kWaveWin;
        next = min(nwin, 2u);
        for (uint32_t win = 0; win < next; ++win) {
            fetch(win, lane);
            store(win, lane);
        }
        if (next < nwin) fetch(next, lane);
    }
    // makes entries up to `last` readable (true when that took a new
    // window); reads advance by less than a window at a time, so the ring
    // slot refilled held a window no longer read
    __device__ bool need(uint32_t last, uint32_t lane) {
        if (last / kWaveWin >= next && next < nwin) {
            store(next, lane);
            ++next;
            if (next < nwin) fetch(next, lane);
            return true;
        }
        return false;
    }
    __device__ T at(uint32_t i) const { return ring[i % kWaveRing]; }
};

// One word column w of one network; rows: LDS of n real plus scratch rows.
// sink: 64 words of LDS, one per lane, that take the idle lanes' accesses.
// With sat, the column stops once every real row is all ones: rows only
// gain bits, so nothing later in the schedule can change it.  It is checked
// whenever a new window of ops enters the ring (every kWaveWin ops, off the
// per-group path), by a scan of the column in LDS that ends at the first
// 64-row block holding a row not yet full.
// W: ops per lane and group; a group is up to 64 * W ops of one level, all
// of whose row reads are issued together (ops of a level are independent).
template <int W>
__device__ void rowor_wave_column(uint64_t *__restrict__ C, int64_t ld, uint32_t n, uint32_t nwords,
                                  const DevOps &s, uint32_t w, uint64_t *rows, uint64_t *sink, op4 *oring,
                                  uint32_t *lring, unsigned long long *__restrict__ traffic, bool sat,
                                  uint32_t *__restrict__ persist, unsigned int *__restrict__ done_count) {
    const uint32_t lane = threadIdx.x;
    const uint32_t rwords = (n + 31) / 32;
    const uint32_t tail = n & 63u;
    const uint64_t fullw = (w + 1 < nwords || tail == 0) ? ~0ull : (1ull << tail) - 1ull;
    uint32_t *pst = persist ? persist + (size_t)w * (2 * (size_t)rwords + 2) : nullptr;
    if (s.L == 0 || s.nops == 0) return;  // nothing to apply: C is left as it is
    if (pst && pst[0]) return;            // the column is all ones already (uniform)
    const uint32_t L = s.L;
    auto slot = [&](uint32_t id) { return (id & kScratchBit) ? n + (id & kNodeMask) : id; };
    WaveRing<op4> opr;
    opr.init(oring, reinterpret_cast<const op4 *>(s.ops), s.nops, lane);
    WaveRing<uint32_t> lvr;
    lvr.init(lring, s.lvl, L + 1, lane);
    auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
    for (uint32_t r = lane; r < n; r += 64) rows[r] = C[(size_t)r * ld + w];
    // group: ops [q0, min(q0 + 64 W, p1)) of level l; p2 = start of level
    // l + 2.  The loop starts on an empty level -1, so that every op and
    // level start it uses was read inside it.
    constexpr uint32_t G = 64 * W;
    uint32_t l = 0xffffffffu, q0 = uni(lvr.at(0)), p1 = q0;
    uint32_t p2 = uni(lvr.at(1));
    uint32_t p3v = L >= 2 ? lvr.at(2) : s.nops;  // start of level l + 3 (lane-uniform VGPR)
    op4 op[W];
#pragma unroll
    for (int k = 0; k < W; ++k) op[k] = op4{0u, 0u, kNoRow, kNoRow};
    for (;;) {
        uint32_t nl = l, nq0, np1, np2 = p2;
        if (q0 + G < p1) {
            nq0 = q0 + G;
            np1 = p1;
        } else {
            nl = l + 1;
            nq0 = p1;
            np1 = p2;
            np2 = uni(p3v);
            if (nl + 3 <= L) {
                lvr.need(nl + 3, lane);
                p3v = lvr.at(nl + 3);
            }
        }
        const bool more = nl < L;
        bool stop = false;
        if (more && np1 > nq0 && opr.need(min(nq0 + G, np1) - 1, lane) && sat) {
            // every group before this one has been applied; this one is
            // applied all the same (it cannot change a full column), so
            // that no path through the loop skips the group's waits
            bool full = true;
            for (uint32_t r0 = 0; r0 < n && full; r0 += 64)
                full = __all(r0 + lane >= n || rows[r0 + lane] == fullw);
            stop = full;
        }
        op4 nop[W];
#pragma unroll
        for (int k = 0; k < W; ++k) nop[k] = opr.at(nq0 + lane + 64 * k);
        {
            // branch-free: idle lanes and absent targets use the lane's own
            // sink word, so every group issues the same LDS operations
            uint64_t *const own = sink + lane;
            bool act[W];
            uint64_t r[W];
#pragma unroll
            for (int k = 0; k < W; ++k) {
                act[k] = q0 + lane + 64 * k < p1;
                r[k] = *(act[k] ? rows + slot(op[k].x) : own) | *(act[k] ? rows + slot(op[k].y) : own);
            }
            // keeps the read of the next group's ops beside the row reads
            // (the compiler would otherwise sink it past the saturation
            // check, a second LDS round trip per group)
#pragma unroll
            for (int k = 0; k < W; ++k)
                asm volatile("" : : "v"(nop[k].x), "v"(nop[k].y), "v"(nop[k].z), "v"(nop[k].w));
#pragma unroll
            for (int k = 0; k < W; ++k) {
                *(act[k] && op[k].z != kNoRow ? rows + slot(op[k].z) : own) = r[k];
                *(act[k] && op[k].w != kNoRow ? rows + slot(op[k].w) : own) = r[k];
            }
        }
        if (!more || stop) break;
#pragma unroll
        for (int k = 0; k < W; ++k) op[k] = nop[k];
        q0 = nq0;
        p1 = np1;
        p2 = np2;
        l = nl;
    }
    for (uint32_t r = lane; r < n; r += 64) C[(size_t)r * ld + w] = rows[r];
    if (traffic && lane == 0) {
        atomicAdd(traffic, (unsigned long long)n);
        atomicAdd(traffic + 1, (unsigned long long)n);
    }
    if (!pst) return;
    int32_t nfull = 0;
    for (uint32_t k = lane; k < rwords; k += 64) {
        uint32_t fb = 0, nz = 0;
        for (uint32_t b = 0; b < 32 && 32 * k + b < n; ++b) {
            const uint64_t v = rows[32 * k + b];
            fb |= (uint32_t)(v == fullw) << b;
            nz |= (uint32_t)(v != 0) << b;
        }
        pst[2 + k] = fb;
        pst[2 + rwords + k] = nz;
        nfull += __popc(fb);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nfull += __shfl_xor(nfull, off);
    if (lane == 0) {
        pst[1] = (uint32_t)nfull;
        if (nfull == (int32_t)n) {
            pst[0] = 1u;
            atomicAdd(done_count, 1u);
        }
    }
}

template <int W>
__global__ void __launch_bounds__(64)
k_rowor_wave(uint64_t *__restrict__ C, int64_t ld, uint32_t n, uint32_t nwords, DevOps s,
             unsigned long long *__restrict__ traffic, bool sat, uint32_t *__restrict__ persist,
             unsigned int *__restrict__ done_count) {
    extern __shared__ uint64_t rows[];  // n real rows, then the scratch rows
    __shared__ op4 oring[kWaveRing];
    __shared__ uint32_t lring[kWaveRing];
    __shared__ uint64_t sink[64];
    rowor_wave_column<W>(C, ld, n, nwords, s, xcd_slice(blockIdx.x, gridDim.x), rows, sink, oring,
                         lring, traffic, sat, persist, done_count);
}

// Many networks of n nodes each (the hashed proxies): wavefront b runs word
// column b % nwords of network b / nwords.
template <int W>
__global__ void __launch_bounds__(64)
k_rowor_wave_multi(const WaveNet *__restrict__ nets, uint32_t n, uint32_t nwords,
                   unsigned long long *__restrict__ traffic, bool sat,
                   unsigned int *__restrict__ done_count) {
    extern __shared__ uint64_t rows[];
    __shared__ op4 oring[kWaveRing];
    __shared__ uint32_t lring[kWaveRing];
    const uint32_t b = xcd_slice(blockIdx.x, gridDim.x);
    const WaveNet &net = nets[b / nwords];
    __shared__ uint64_t sink[64];
    rowor_wave_column<W>(net.C, net.ld, n, nwords, net.s, b % nwords, rows, sink, oring, lring,
                         traffic, sat, net.persist, done_count);
}

// The same stream from a flat schedule (many networks of n nodes, one
// wavefront per word column): ops in level order, their rows as LDS byte
// offsets of the column (kFlatNone: no second target) and bit 31 of the
// first offset set on the last op of every level.  A group is up to 64 ops
// of one level; the next group's ops are read ahead, and one ballot of
// their level-end bits gives its size, so the loop keeps no level starts.
// Word column w of one network with a flat schedule (one wavefront).
__device__ __forceinline__ void
rowor_wave_flat_column(const WaveNet &net, uint32_t w, uint32_t n, uint32_t nwords, bool sat,
                       unsigned int *__restrict__ done_count,
                       unsigned long long *__restrict__ traffic) {
    extern __shared__ uint64_t rows[];
    __shared__ op4 oring[kWaveRing];
    __shared__ uint64_t sink[64];
    const uint32_t lane = threadIdx.x;
    const uint32_t rwords = (n + 31) / 32;
    const uint32_t tail = n & 63u;
    const uint64_t fullw = (w + 1 < nwords || tail == 0) ? ~0ull : (1ull << tail) - 1ull;
    uint32_t *pst = net.persist ? net.persist + (size_t)w * (2 * (size_t)rwords + 2) : nullptr;
    const uint32_t nops = net.s.nops;
    if (nops == 0) return;       // nothing to apply: C is left as it is
    if (pst && pst[0]) return;   // the column is all ones already (uniform)
    uint64_t *const C = net.C;
    const int64_t ld = net.ld;
    for (uint32_t r = lane; r < n; r += 64) rows[r] = C[(size_t)r * ld + w];
    WaveRing<op4> opr;
    opr.init(oring, reinterpret_cast<const op4 *>(net.s.ops), nops, lane);
    unsigned char *const base = reinterpret_cast<unsigned char *>(rows);
    uint64_t *const own = sink + lane;
    auto row = [&](uint32_t off) { return reinterpret_cast<uint64_t *>(base + (off & kFlatOffMask)); };
    auto group = [&](const op4 &o, uint32_t q) -> uint32_t {
        const uint64_t ends = __ballot(q + lane < nops && (o.x >> 31));
        const uint32_t g = ends ? (uint32_t)__ffsll((unsigned long long)ends) : 64u;
        return min(g, nops - q);
    };
    uint32_t q = 0;
    op4 op = opr.at(lane);
    uint32_t size = group(op, 0);
    for (;;) {
        const uint32_t nq = q + size;
        const bool more = nq < nops;
        bool stop = false;
        if (more && opr.need(min(nq + 64, nops) - 1, lane) && sat) {
            // every group before this one has been applied; this one is
            // applied all the same (it cannot change a full column)
            bool full = true;
            for (uint32_t r0 = 0; r0 < n && full; r0 += 64)
                full = __all(r0 + lane >= n || rows[r0 + lane] == fullw);
            stop = full;
        }
        const op4 nop = opr.at(nq + lane);
        {
            const bool act = lane < size;
            const uint64_t r = *(act ? row(op.x) : own) | *(act ? row(op.y) : own);
            asm volatile("" : : "v"(nop.x), "v"(nop.y), "v"(nop.z), "v"(nop.w));
            *(act && op.z != kFlatNone ? row(op.z) : own) = r;
            *(act && op.w != kFlatNone ? row(op.w) : own) = r;
        }
        if (!more || stop) break;
        size = group(nop, nq);
        op = nop;
        q = nq;
    }
    for (uint32_t r = lane; r < n; r += 64) C[(size_t)r * ld + w] = rows[r];
    if (traffic && lane == 0) {
        atomicAdd(traffic, (unsigned long long)n);
        atomicAdd(traffic + 1, (unsigned long long)n);
    }
    if (!pst) return;
    int32_t nfull = 0;
    for (uint32_t k = lane; k < rwords; k += 64) {
        uint32_t fb = 0, nz = 0;
        for (uint32_t bb = 0; bb < 32 && 32 * k + bb < n; ++bb) {
            const uint64_t v = rows[32 * k + bb];
            fb |= (uint32_t)(v == fullw) << bb;
            nz |= (uint32_t)(v != 0) << bb;
        }
        pst[2 + k] = fb;
        pst[2 + rwords + k] = nz;
        nfull += __popc(fb);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nfull += __shfl_xor(nfull, off);
    if (lane == 0) {
        pst[1] = (uint32_t)nfull;
        if (nfull == (int32_t)n) {
            pst[0] = 1u;
            atomicAdd(done_count, 1u);
        }
    }
}

// count networks (nets: device array), one block per (network, column)
__global__ void __launch_bounds__(64)
k_rowor_wave_flat(const WaveNet *__restrict__ nets, uint32_t n, uint32_t nwords, bool sat,
                  unsigned int *__restrict__ done_count,
                  unsigned long long *__restrict__ traffic) {
    const uint32_t b = xcd_slice(blockIdx.x, gridDim.x);
    rowor_wave_flat_column(nets[b / nwords], b % nwords, n, nwords, sat, done_count, traffic);
}

// one network passed by value (a resident plan), one block per column
__global__ void __launch_bounds__(64)
k_rowor_wave_flat1(WaveNet net, uint32_t n, uint32_t nwords, bool sat,
                   unsigned long long *__restrict__ traffic) {
    rowor_wave_flat_column(net, xcd_slice(blockIdx.x, gridDim.x), n, nwords, sat, nullptr,
                           traffic);
}

}  // namespace

size_t flat_ops_bytes(const HostSchedule &s) { return std::max<size_t>(256, 4 * s.ops.size()); }

void flat_ops_pack(const HostSchedule &s, uint32_t n, uint32_t *out) {
    auto byte_off = [n](uint32_t id) -> uint32_t {
        return 8u * ((id & kScratchBit) ? n + (id & kNodeMask) : id);
    };
    for (uint32_t l = 0; l < s.Lops; ++l) {
        const uint32_t q1 = s.lvl_op[l + 1];
        for (uint32_t q = s.lvl_op[l]; q < q1; ++q) {
            const uint32_t *src = &s.ops[4 * (size_t)q];
            uint32_t *o = out + 4 * (size_t)q;
            o[0] = byte_off(src[0]) | (q + 1 == q1 ? kFlatEnd : 0u);
            o[1] = byte_off(src[1]);
            o[2] = src[2] == kNoRow ? kFlatNone : byte_off(src[2]);
            o[3] = src[3] == kNoRow ? kFlatNone : byte_off(src[3]);
        }
    }
}

hipError_t launch_rowor_wave_flat(const WaveNet *nets, uint32_t count, uint32_t n,
                                  uint32_t max_scratch_rows, bool saturation,
                                  unsigned int *done_count, unsigned long long *traffic,
                                  hipStream_t st) {
    if (count == 0) return hipSuccess;
    if (!rowor_wave_fits(n, max_scratch_rows)) return hipErrorInvalidValue;
    const uint32_t nwords = (n + 63) / 64;
    const size_t lds = ((size_t)n + max_scratch_rows + 1) * 8;
    hipError_t e = hipFuncSetAttribute((const void *)k_rowor_wave_flat,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rowor_wave_flat, dim3(count * nwords), dim3(64), lds, st, nets, n, nwords,
                       saturation, done_count, traffic);
    return hipGetLastError();
}

hipError_t launch_rowor_wave_flat1(const uint32_t *flat_ops, uint32_t nops, uint32_t n,
                                   uint64_t *C, int64_t ld, uint32_t scratch_rows,
                                   unsigned long long *traffic, bool saturation, hipStream_t st) {
    if (nops == 0) return hipSuccess;
    if (!rowor_wave_fits(n, scratch_rows)) return hipErrorInvalidValue;
    const uint32_t nwords = (n + 63) / 64;
    const size_t lds = ((size_t)n + scratch_rows + 1) * 8;
    hipError_t e = hipFuncSetAttribute((const void *)k_rowor_wave_flat1,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    WaveNet net{};
    net.s.nops = nops;
    net.s.ops = reinterpret_cast<const uint4 *>(flat_ops);
    net.C = C;
    net.ld = ld;
    hipLaunchKernelGGL(k_rowor_wave_flat1, dim3(nwords), dim3(64), lds, st, net, n, nwords,
                       saturation, traffic);
    return hipGetLastError();
}

bool rowor_wave_fits(uint32_t n, uint32_t scratch_rows) {
    return ((size_t)n + scratch_rows + 1) * 8 <= kRoworWaveLds;
}

bool rowor_wave_pays(uint32_t n, uint32_t scratch_rows, int64_t ops, int64_t levels) {
    return rowor_wave_fits(n, scratch_rows) && ops <= kRoworWaveOpsPerLevel * levels;
}

hipError_t launch_rowor_wave(const DevOps &s, uint32_t n, uint64_t *C, int64_t ld,
                             uint32_t scratch_rows, unsigned long long *traffic, bool saturation,
                             uint32_t *persist, unsigned int *done_count, hipStream_t st) {
    if (s.L == 0 || s.nops == 0) return hipSuccess;
    if (!rowor_wave_fits(n, scratch_rows)) return hipErrorInvalidValue;
    const uint32_t nwords = (n + 63) / 64;
    const size_t lds = ((size_t)n + scratch_rows + 1) * 8;
    const bool wide = rowor_wave_wide(s.nops, s.L);
    const void *fn = wide ? (const void *)k_rowor_wave<2> : (const void *)k_rowor_wave<1>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (wide)
        hipLaunchKernelGGL(k_rowor_wave<2>, dim3(nwords), dim3(64), lds, st, C, ld, n, nwords, s,
                           traffic, saturation, persist, done_count);
    else
        hipLaunchKernelGGL(k_rowor_wave<1>, dim3(nwords), dim3(64), lds, st, C, ld, n, nwords, s,
                           traffic, saturation, persist, done_count);
    return hipGetLastError();
}

hipError_t launch_rowor_wave_multi(const WaveNet *nets, uint32_t count, uint32_t n,
                                   uint32_t max_scratch_rows, bool wide,
                                   unsigned long long *traffic, bool saturation,
                                   unsigned int *done_count, hipStream_t st) {
    if (count == 0) return hipSuccess;
    if (!rowor_wave_fits(n, max_scratch_rows)) return hipErrorInvalidValue;
    const uint32_t nwords = (n + 63) / 64;
    const size_t lds = ((size_t)n + max_scratch_rows + 1) * 8;
    const void *fn = wide ? (const void *)k_rowor_wave_multi<2> : (const void *)k_rowor_wave_multi<1>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (wide)
        hipLaunchKernelGGL(k_rowor_wave_multi<2>, dim3(count * nwords), dim3(64), lds, st, nets, n,
                           nwords, traffic, saturation, done_count);
    else
        hipLaunchKernelGGL(k_rowor_wave_multi<1>, dim3(count * nwords), dim3(64), lds, st, nets, n,
                           nwords, traffic, saturation, done_count);
    return hipGetLastError();
}

bool rowor_wave_wide(int64_t ops, int64_t levels) { return ops > kRoworWaveWideOps * levels; }

}  // namespace tn
