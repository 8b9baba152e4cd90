// gfx950 kernels of the exact component-matrix path.
//
// The matrix is n rows of ld uint64 words; row u is the out-component of u
// (Sec. 3.1, stored transposed so the reverse-time update of Sec. 3.4 ORs
// rows).  Every update only ORs words of one column range into the same
// column range of another row, so each word column evolves on its own: a
// workgroup that owns a slice of word columns of every row can run all levels
// of the schedule with workgroup barriers only, and no two workgroups ever
// touch the same word.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tn_device.h"
#include "tn_internal.h"

namespace tn {

namespace {

__global__ void __launch_bounds__(256) k_identity(uint64_t *__restrict__ C, uint32_t n, int64_t ld,
                                                  unsigned long long *__restrict__ traffic) {
    if (traffic && blockIdx.x == 0 && threadIdx.x < 2) traffic[threadIdx.x] = 0;
    for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
        uint64_t *row = C + (size_t)r * (size_t)ld;
        const int64_t diag = (int64_t)(r >> 6);
        const uint64_t bit = 1ull << (r & 63u);
        for (int64_t j = threadIdx.x; j < ld; j += blockDim.x) row[j] = (j == diag) ? bit : 0ull;
    }
}

// One workgroup per slice of SW word columns runs every level of the
// binary-op schedule; SW consecutive lanes update the SW words of one op's
// rows, so each row access is one contiguous 8*SW-byte segment.  An op is
// r = row[a] | row[b]; row[d1] = r; row[d2] = r: an undirected pair is
// (u, v, u, v), a one-way pair (u, v, u, -), and a compound time step folds
// its old rows into scratch rows and copies them back, so every level is the
// same straight-line code over at most kOpsLevelCap independent ops.
//
// Saturation.  Rows only gain bits in reverse time, and once an
// out-component covers every column of a slice, any OR with it is that full
// slice again.  With SAT, each workgroup keeps one LDS bit per row (and per
// scratch row) meaning "this row is all ones in my slice".  An op with a
// saturated operand loads nothing and gives a full result; a store of a full
// result into a row already marked full is dropped.  Every write refreshes
// the destination's bit, so a bit of 1 is always true (0 only means "not
// known"), and the matrix in memory is exactly the plain recurrence's.
// Kernel counters record the row words actually loaded and stored.
//
// The waves of a workgroup specialise.  Two loader waves stream the ops of
// level l + 1 into an LDS frame while the compute waves run level l from the
// other frame; the ops of levels l + 2 and l + 3 are already in flight into
// the loaders' registers.
// Compute waves issue only row loads and stores.  On gfx9 loads and stores
// share one in-order completion counter, so this split keeps the loaders'
// waits from ever covering row stores, and the compute waves never wait for
// a schedule load.  A row access is issued only by the lanes that need it
// (exec-masked): a lane aimed at a sink word instead costs the CU's texture
// address and data units, which bound these kernels, as much as a real
// access.  The barrier that ends a level orders the workgroup's row stores
// and bit updates before the next level.
constexpr uint32_t kLoaderThreads = 128;
constexpr uint32_t kLoaderOps = kOpsLevelCap / kLoaderThreads;  // ops per loader lane and level
constexpr uint32_t kFrames = 2;  // LDS op frames: the level being run and the next


struct OpArgs {
    uint64_t *C;
    size_t ldz;
    uint64_t *rows;  // scratch rows of nwords words, sld apart
    uint64_t *sink;  // this thread's sink word
    uint32_t w, nwords, grp, ngrp;
    bool wok;
    // saturation bits (SAT only)
    uint32_t *sat;      // LDS bitmap: real rows from bit 0, scratch rows from bit sbase
    uint32_t sbase;     // first bit of the scratch rows (n rounded up to 32)
    uint32_t sbits;     // bits in the bitmap
    uint64_t fullw;     // this lane's word when its row slice is full (0 past the last word)
    uint64_t gmask;     // ballot bits of this lane's group
    int32_t *nfull;           // this level's change of the full real-row count
    int32_t dfull, dzero;     // this lane's part of those changes, added once per wave
    // zero bits (word-range skipping): same indexing as the saturation bits,
    // bit set = the row is all zero in this slice
    uint32_t *zb;
    int32_t *nzero;           // this level's change of the zero real-row count
    bool zon;                 // some real row is still zero (uniform per level)
    uint32_t loaded, stored;  // row words this lane moved
    bool lead;                // first lane of its group
    uint32_t ld32;            // ldz, for 32-bit row offsets (fwd_addr)
    uint32_t sld;             // scratch row stride: nwords rounded up to even
    uint32_t vw;              // row words this lane covers (two-word lanes)
    uint64_t fullw1;          // fullw of the lane's second word (two-word lanes)
};

// The lane's full row-slice value.
template <int LW>
__device__ __forceinline__ typename LaneT<LW>::T lane_full(const OpArgs &A) {
    if constexpr (LW == 1) {
        return A.fullw;
    } else {
        return u64x2{A.fullw, A.fullw1};
    }
}
// Clears a two-word lane's word past the row's last one (padding).
template <int LW>
__device__ __forceinline__ typename LaneT<LW>::T lane_keep(const OpArgs &A) {
    if constexpr (LW == 1) {
        return ~0ull;
    } else {
        return u64x2{~0ull, A.w + 1 < A.nwords ? ~0ull : 0ull};
    }
}

// The address of a row or scratch row word, chosen without a branch (the
// lane's sink word where not valid).
__device__ __forceinline__ uint64_t *op_addr(const OpArgs &A, uint32_t id, bool valid) {
    const uint64_t row = (uint64_t)(id & kNodeMask);
    const uintptr_t real = (uintptr_t)(A.C + row * A.ldz + A.w);
    const uintptr_t scr = (uintptr_t)(A.rows + row * A.sld + A.w);
    const uintptr_t pick = (id & kScratchBit) ? scr : real;
    const bool ok = valid && A.wok && id != kNoRow;
    return (uint64_t *)(ok ? pick : (uintptr_t)A.sink);
}

// op_addr with 32-bit row offsets: a 24-bit multiply instead of 64-bit
// ones, when rows and strides are below 2^24 and every offset below 2^32
// (the host checks; rowor_fwd_off32).
template <bool OFF32>
__device__ __forceinline__ uint64_t *fwd_addr(const OpArgs &A, uint32_t id, bool valid) {
    if (!OFF32) return op_addr(A, id, valid);
    const bool scr = id & kScratchBit;
    const uint32_t off = __umul24(id & kNodeMask, scr ? A.sld : A.ld32) + A.w;
    uint64_t *base = scr ? A.rows : A.C;
    const bool ok = valid && A.wok && id != kNoRow;
    return ok ? base + off : A.sink;
}

__device__ __forceinline__ uint32_t sat_index(const OpArgs &A, uint32_t id) {
    const uint32_t i = (id & kScratchBit) ? A.sbase + (id & kNodeMask) : id;
    return min(i, A.sbits - 1);  // kNoRow and stale frame entries stay in range
}

__device__ __forceinline__ bool sat_get(const OpArgs &A, uint32_t id) {
    const uint32_t i = sat_index(A, id);
    return (A.sat[i >> 5] >> (i & 31u)) & 1u;
}

__device__ __forceinline__ bool zero_get(const OpArgs &A, uint32_t id) {
    const uint32_t i = sat_index(A, id);
    return (A.zb[i >> 5] >> (i & 31u)) & 1u;
}

// A real row leaves the zero set once and never returns (rows only gain
// bits); a scratch row is zero or not after each store into it.
__device__ __forceinline__ void zero_set(OpArgs &A, uint32_t id, bool zero) {
    const uint32_t i = sat_index(A, id);
    if (zero) atomicOr(&A.zb[i >> 5], 1u << (i & 31u));
    else atomicAnd(&A.zb[i >> 5], ~(1u << (i & 31u)));
    if (!(id & kScratchBit)) A.dzero += zero ? 1 : -1;
}

// Plain path: ops [base, n) of the current frame, UC per lane group, every
// op loading and storing its rows; MAX8 merges rows by byte-wise maximum
// instead of OR.
template <int UC, bool MAX8 = false>
__device__ __forceinline__ void apply_frame(OpArgs &A, const op4 *frame, uint32_t base,
                                            uint32_t n) {
    op4 o[UC];
    uint64_t x[UC], y[UC];
#pragma unroll
    for (int k = 0; k < UC; ++k) o[k] = frame[min(base + A.grp + k * A.ngrp, kOpsLevelCap - 1)];
    // only lanes with a row to move access memory (see fwd_issue)
#pragma unroll
    for (int k = 0; k < UC; ++k) {
        const bool v = base + A.grp + k * A.ngrp < n && A.wok;
        x[k] = y[k] = 0ull;
        if (v) x[k] = *op_addr(A, o[k].x, true);
        if (v) y[k] = *op_addr(A, o[k].y, true);
        A.loaded += v ? 2u : 0u;
    }
#pragma unroll
    for (int k = 0; k < UC; ++k) {
        const bool v = base + A.grp + k * A.ngrp < n && A.wok;
        const uint64_t r = MAX8 ? max_bytes7(x[k], y[k]) : (x[k] | y[k]);
        if (v && o[k].z != kNoRow) *op_addr(A, o[k].z, true) = r;
        if (v && o[k].w != kNoRow) *op_addr(A, o[k].w, true) = r;
        A.stored += ((v && A.wok && o[k].z != kNoRow) ? 1u : 0u) +
                    ((v && A.wok && o[k].w != kNoRow) ? 1u : 0u);
    }
}

// Saturation path, per compute wave: classify a contiguous share of the
// level's ops by their saturation bits (LDS only), keep those that still
// need a row load or store in a per-wave list (ballot compaction), then run
// only those.
constexpr uint32_t kComputeWaves = (1024 - kLoaderThreads) / 64;
constexpr uint32_t kWaveShare = (kOpsLevelCap + kComputeWaves - 1) / kComputeWaves;
constexpr uint32_t kWorkSkip = 1u << 16, kWorkF1 = 1u << 17, kWorkF2 = 1u << 18;
// zero flags: the result is zero (no loads), an operand is zero (no load
// of it), a destination is zero
constexpr uint32_t kWorkZero = 1u << 19, kWorkZX = 1u << 20, kWorkZY = 1u << 21;
constexpr uint32_t kWorkZ1 = 1u << 22, kWorkZ2 = 1u << 23;

// Flips the bit of a row whose state changed; a real row also moves this
// lane's part of the level's count of full real rows, added once per wave
// (level_counts).
__device__ __forceinline__ void sat_set(OpArgs &A, uint32_t id, bool full) {
    const uint32_t i = sat_index(A, id);
    if (full) atomicOr(&A.sat[i >> 5], 1u << (i & 31u));
    else atomicAnd(&A.sat[i >> 5], ~(1u << (i & 31u)));
    if (!(id & kScratchBit)) A.dfull += full ? 1 : -1;
}

// Adds the wave's changes of the full and zero real-row counts, kept per
// lane over the level, to this level's LDS counters: the compiler combines
// the lanes of one atomic (a scalar loop over the lanes with a change) into
// a single LDS atomic per wave and counter, where one atomic per row change
// would serialize on the one address.  A shuffle reduction instead costs a
// dozen dependent LDS permutes on every wave with a change (0.18 us more
// per level of the saturating rest with 1-50 work items).
__device__ __forceinline__ void level_counts(OpArgs &A) {
    if (A.dfull) atomicAdd(A.nfull, A.dfull);
    if (A.dzero) atomicAdd(A.nzero, A.dzero);
    A.dfull = A.dzero = 0;
}

// The wave's nwork items (wave-uniform), one per lane group at a time.
// Batching several items' loads per lane before their stores measured
// slower, both where most ops still need rows and in the sparse tail, where
// one pass of U items per lane group took 5.6 us per busy level against
// 5.1 us and 1.7 us per one-item level against 1.1 us (the idle items' sink
// stores): a busy level is bound by the workgroup's memory throughput, not
// by serialized round trips.
template <int SW, bool ZERO, int LW>
__device__ __forceinline__ void run_work(OpArgs &A, const op4 *frame, const uint32_t *work,
                                         uint32_t nwork) {
    using T = typename LaneT<LW>::T;
    constexpr uint32_t SL = SW / LW;  // lanes per op
    constexpr uint32_t G = 64 / SL;   // lane groups per wave
    const uint32_t g = (threadIdx.x & 63u) / SL;
    const T fullv = lane_full<LW>(A);
    for (uint32_t j0 = 0; j0 < nwork; j0 += G) {
        const uint32_t j = j0 + g;
        const uint32_t e = work[min(j, kWaveShare - 1)];
        const op4 o = frame[e & (kOpsLevelCap - 1)];
        const bool v = j < nwork, skip = e & kWorkSkip;
        const bool f1 = e & kWorkF1, f2 = e & kWorkF2;
        if (__ballot(v && !skip) == 0) {
            // Every item of the batch has a full operand, so every result is
            // the full slice: nothing is read, and the stores take the full
            // word, whose register nothing overwrites.  (A store's data
            // register may not be rewritten before the store retires, and
            // loads and stores retire in order: a result register rewritten
            // item after item, or a wait for a load, would wait for every
            // earlier store of the wave.)  Most batches look like this once
            // most rows are full.
            const bool s1 = v && o.z != kNoRow && !f1;
            const bool s2 = v && o.w != kNoRow && !f2;
            if (s1 && A.wok) *(T *)op_addr(A, o.z, true) = fullv;
            if (s2 && A.wok) *(T *)op_addr(A, o.w, true) = fullv;
            A.stored += (s1 ? A.vw : 0u) + (s2 ? A.vw : 0u);
            if (v && A.lead) {
                if (s1) sat_set(A, o.z, true);
                if (s2) sat_set(A, o.w, true);
                if (ZERO && A.zon) {
                    if (o.z != kNoRow && (e & kWorkZ1)) zero_set(A, o.z, false);
                    if (o.w != kNoRow && (e & kWorkZ2)) zero_set(A, o.w, false);
                }
            }
            continue;
        }
        // an operand known zero in this slice is not loaded
        const bool ldx = v && !skip && !(ZERO && (e & (kWorkZero | kWorkZX)));
        const bool ldy = v && !skip && !(ZERO && (e & (kWorkZero | kWorkZY)));
        const T none = T(0);
        T r = skip ? fullv : none;
        if (__ballot(ldx || ldy) != 0) {
            T x = none, y = none;
            if (ldx && A.wok) x = *(const T *)op_addr(A, o.x, true);
            if (ldy && A.wok) y = *(const T *)op_addr(A, o.y, true);
            A.loaded += (ldx ? A.vw : 0u) + (ldy ? A.vw : 0u);
            // a word past the row's last one (two-word lanes) is padding:
            // its full value is zero, and it is kept zero
            if (!skip) r = ((ldx ? x : none) | (ldy ? y : none)) & lane_keep<LW>(A);
        }
        // the group's lanes agree on whether the whole row slice is full
        const uint64_t ball = __ballot(lane_eq<LW>(r, fullv) || !A.wok);
        const bool full = (ball & A.gmask) == A.gmask;
        bool zero = false;
        if (ZERO && A.zon) {
            const uint64_t zb = __ballot(lane_eq<LW>(r, none) || !A.wok);
            zero = (zb & A.gmask) == A.gmask;
        }
        const bool z1 = ZERO && (e & kWorkZ1), z2 = ZERO && (e & kWorkZ2);
        // a full result into a full row, or a zero result into a zero row,
        // changes nothing
        const bool s1 = v && o.z != kNoRow && !(full && f1) && !(zero && z1);
        const bool s2 = v && o.w != kNoRow && !(full && f2) && !(zero && z2);
        if (s1 && A.wok) *(T *)op_addr(A, o.z, true) = r;
        if (s2 && A.wok) *(T *)op_addr(A, o.w, true) = r;
        A.stored += (s1 ? A.vw : 0u) + (s2 ? A.vw : 0u);
        // one lane per group refreshes the destinations' bits
        if (v && A.lead) {
            if (o.z != kNoRow && f1 != full) sat_set(A, o.z, full);
            if (o.w != kNoRow && f2 != full) sat_set(A, o.w, full);
            if (ZERO && A.zon) {
                if (o.z != kNoRow && z1 != zero) zero_set(A, o.z, zero);
                if (o.w != kNoRow && z2 != zero) zero_set(A, o.w, zero);
            }
        }
    }
}

// Classify ops [lo, hi) of the frame (hi - lo <= kWaveShare) into this
// wave's work list; returns the list length (wave-uniform).
// With ZERO and while some real row is zero, an op whose operands are both
// zero has a zero result; it still needs a store only into a destination not
// known to be zero (a scratch row: a real destination is contained in the
// result, so it is zero too).
template <bool ZERO>
__device__ __forceinline__ uint32_t classify(const OpArgs &A, const op4 *frame, uint32_t lo,
                                             uint32_t hi, uint32_t *work) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t nwork = 0;
    for (uint32_t r0 = lo; r0 < hi; r0 += 64) {
        const uint32_t i = r0 + lane;
        const bool v = i < hi;
        const op4 o = frame[min(i, kOpsLevelCap - 1)];
        // every bit read is issued at once (no short-circuit: one LDS round
        // trip, not four; sat_index keeps kNoRow in range)
        const bool skip = sat_get(A, o.x) | sat_get(A, o.y);
        const bool f1 = (o.z != kNoRow) & sat_get(A, o.z);
        const bool f2 = (o.w != kNoRow) & sat_get(A, o.w);
        bool zx = false, zy = false, z1 = false, z2 = false;
        if (ZERO && A.zon) {
            zx = zero_get(A, o.x);
            zy = zero_get(A, o.y);
            z1 = (o.z != kNoRow) & zero_get(A, o.z);
            z2 = (o.w != kNoRow) & zero_get(A, o.w);
        }
        const bool zres = !skip && zx && zy;
        const bool need =
            v && (skip ? ((o.z != kNoRow && !f1) || (o.w != kNoRow && !f2))
                       : (!zres || (o.z != kNoRow && !z1) || (o.w != kNoRow && !z2)));
        const uint64_t m = __ballot(need);
        const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (need)
            work[nwork + pos] = i | (skip ? kWorkSkip : 0u) | (f1 ? kWorkF1 : 0u) |
                                (f2 ? kWorkF2 : 0u) | (zres ? kWorkZero : 0u) |
                                (zx ? kWorkZX : 0u) | (zy ? kWorkZY : 0u) |
                                (z1 ? kWorkZ1 : 0u) | (z2 ? kWorkZ2 : 0u);
        nwork += (uint32_t)__popcll(m);
    }
    return nwork;
}

// Loader lanes hold a level's ops in registers.
struct HeldOps {
    op4 r[kLoaderOps];
};

// The ops of the level that starts at op p0 into registers (clamped,
// unconditional).
__device__ __forceinline__ HeldOps fetch_ops(const DevOps &s, uint32_t p0, uint32_t lane) {
    const uint32_t last = s.nops - 1;
    const op4 *ops = reinterpret_cast<const op4 *>(s.ops);
    HeldOps h;
#pragma unroll
    for (int k = 0; k < (int)kLoaderOps; ++k) h.r[k] = ops[min(p0 + lane + k * kLoaderThreads, last)];
    return h;
}

// First op of level l (l clamped to L, whose entry is nops).
__device__ __forceinline__ uint32_t level_start(const DevOps &s, uint32_t l) {
    return s.lvl[min(l, s.L)];
}

__device__ __forceinline__ void put_level(op4 *frame, const HeldOps &h, uint32_t lane) {
#pragma unroll
    for (int k = 0; k < (int)kLoaderOps; ++k) frame[lane + k * kLoaderThreads] = h.r[k];
}

// Wave sum of a per-lane count, added once per wave to a device counter.
__device__ __forceinline__ void count_add(unsigned long long *ctr, uint32_t x) {
    unsigned long long v = x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63u) == 0 && v) atomicAdd(ctr, v);
}

// The level loop of k_rowor_global over the levels of s, on loader and
// compute waves (A, nfull and nzero set up by the caller); returns, on the
// compute waves, whether the slice stopped with every real row full (then
// nfull is n), else nfull after the last level.  Loader waves return after
// their loop.
template <int SW, int UC, bool SAT, bool MAX8, bool ZERO, int LW>
__device__ __forceinline__ bool level_loop(OpArgs &A, const DevOps &s, uint32_t n, bool loader,
                                           uint32_t tid, uint32_t ctid,
                                           op4 (*frame)[kOpsLevelCap], uint32_t *fcount,
                                           uint32_t (*worklist)[kWaveShare], int32_t *fdelta,
                                           int32_t *zdelta, int32_t &nfull, int32_t &nzero) {
    const uint32_t L = s.L;
    // all waves add the same deltas at the same barriers, so they agree
    // A slice may stop only at the start of a level that is a multiple of 3:
    // the loaders' loop, unrolled by three, then has one exit, at the top (an
    // exit after each level's feed let the compiler's waits in that loop
    // drain the loads of the levels ahead).  Both loops run to L rounded up
    // to a multiple of 3; the levels past L have no ops.  done(l) must be
    // called once for every level, after the barrier that ends level l - 1.
    const uint32_t L3 = (L + 2) / 3 * 3;
    auto done = [&](uint32_t l) -> bool {
        if (!SAT) return false;
        // the delta of level l - 1 (slot 2 is still zero at level 0): read
        // unconditionally, beside the level's other LDS reads
        nfull += fdelta[(l + 2) % 3];
        return l % 3 == 0 && nfull == (int32_t)n;
    };
    constexpr bool WIDE = ((1024 - kLoaderThreads) / SW) * UC < kOpsLevelCap;
    // Loader and compute waves run separate loops with one barrier per level
    // each (the branch is uniform per wave, and s_barrier only counts
    // waves), so the compiler tracks the loaders' loads apart from the
    // compute waves' row traffic.  Loader waves keep three levels in flight
    // in registers (hA, hB, hC): a schedule load has three level periods to
    // land before its frame is written.  Their loop is unrolled by three so
    // that the sets never change registers (a register copy would wait for
    // the load).
    if (loader) {
        // Every loader lane reads the level starts too (the same address in
        // all lanes); a start is loaded one level before the ops it locates,
        // and ahead of them, so each wait below leaves the newer loads in
        // flight.
        uint32_t p1 = level_start(s, 1), p2 = level_start(s, 2), p3 = level_start(s, 3);
        put_level(frame[0], fetch_ops(s, level_start(s, 0), tid), tid);
        if (tid == 0) fcount[0] = p1 - level_start(s, 0);
        HeldOps hA = fetch_ops(s, p1, tid);
        HeldOps hB = fetch_ops(s, p2, tid);
        uint32_t p4 = level_start(s, 4);
        HeldOps hC = fetch_ops(s, p3, tid);
        __syncthreads();
        // at level l: h holds the ops of level l + 1, fetched three levels
        // before (a level whose ops need no memory takes less than a memory
        // round trip, so two levels of lead were not enough); p1..p4 the
        // starts of levels l + 1 .. l + 4
        auto feed = [&](uint32_t l, HeldOps &h) {
            // past the last level frames and counts are never read, and the
            // level starts clamp to L
            const uint32_t nf = (l + 1) % kFrames;
            put_level(frame[nf], h, tid);
            if (tid == 0) fcount[nf] = p2 - p1;
            const uint32_t q = p4;
            p1 = p2;
            p2 = p3;
            p3 = q;
            h = fetch_ops(s, q, tid);
            __syncthreads();
            // after the barrier, so that its latency overlaps the next
            // level's frame writes: issued before it, the wait for those LDS
            // writes at the barrier would wait for this load too (scalar
            // loads and LDS share one counter)
            p4 = level_start(s, l + 5);
        };
        for (uint32_t l = 0; l < L3; l += 3) {
            if (done(l)) break;
            feed(l, hA);
            (void)done(l + 1);  // counts only: not a multiple of 3
            feed(l + 1, hB);
            (void)done(l + 2);
            feed(l + 2, hC);
        }
        return false;
    }
    __syncthreads();
    bool stopped = false;
    for (uint32_t l = 0; l < L3; ++l) {
        const uint32_t cf = l % kFrames;
        const uint32_t cnt = fcount[cf];
        if (done(l)) {
            stopped = true;
            break;
        }
        if (SAT) {
            A.nfull = &fdelta[l % 3];
            if (ctid == 0) fdelta[(l + 1) % 3] = 0;
            if (ZERO) {
                // the zero count settles like the full count: every compute
                // wave adds the same delta after the same barrier
                if (l > 0) nzero += zdelta[(l - 1) % 3];
                A.nzero = &zdelta[l % 3];
                if (ctid == 0) zdelta[(l + 1) % 3] = 0;
                A.zon = nzero > 0;
            }
            const uint32_t cw = ctid >> 6;
            const uint32_t share = (cnt + kComputeWaves - 1) / kComputeWaves;
            const uint32_t lo = min(cw * share, cnt), hi = min(lo + share, cnt);
            uint32_t *work = worklist[SAT ? cw : 0];
            run_work<SW, ZERO, LW>(A, frame[cf], work, classify<ZERO>(A, frame[cf], lo, hi, work));
            level_counts(A);
        } else {
            apply_frame<UC, MAX8>(A, frame[cf], 0, cnt);
            if (WIDE) {
                const uint32_t chunk = A.ngrp * UC;
                for (uint32_t base = chunk; base < cnt; base += chunk)
                    apply_frame<UC, MAX8>(A, frame[cf], base, cnt);
            }
        }
        __syncthreads();
    }
    // the last level's delta settled at the loop's final barrier
    if (SAT && !stopped) nfull += fdelta[(L3 - 1) % 3];
    return stopped;
}

// CHUNK: one launch per chunk of a streamed build, with the slice state in
// `persist` (a separate instantiation, so traces and counters keep the two
// kinds of launch apart).
// LW words per lane (2: 16-byte row accesses, saturating launches only;
// rows must start on 16 bytes).
template <int SW, int UC, bool SAT, bool CHUNK, bool MAX8 = false, bool ZERO = false, int LW = 1>
__global__ void __launch_bounds__(1024)
k_rowor_global(uint64_t *__restrict__ C, int64_t ld, uint32_t n, uint32_t nwords, DevOps s,
               uint64_t *__restrict__ scratch, uint64_t *__restrict__ rows, uint32_t sbase,
               uint32_t sbits, unsigned long long *__restrict__ traffic,
               uint32_t *__restrict__ persist, unsigned int *__restrict__ done_count,
               const uint32_t *__restrict__ order) {
    __shared__ op4 frame[kFrames][kOpsLevelCap];
    __shared__ uint32_t fcount[kFrames];
    __shared__ uint32_t worklist[SAT ? kComputeWaves : 1][kWaveShare];
    // change of the number of full real rows in levels l, l+1, l+2 (mod 3):
    // level l adds into slot l % 3, every wave reads it after the barrier
    // that ends level l, and slot (l + 1) % 3 is cleared during level l
    __shared__ int32_t fdelta[3];
    // the same for the zero real-row count (ZERO), and its start value
    __shared__ int32_t zdelta[3];
    __shared__ int32_t zcount0;
    // dynamic: the saturation bitmap, then (ZERO) the zero bitmap
    extern __shared__ uint32_t satbits[];
    const uint32_t L = s.L;
    if (L == 0 || s.nops == 0) return;
    const uint32_t tid = threadIdx.x;
    const bool loader = tid < kLoaderThreads;
    const uint32_t ctid = tid - kLoaderThreads;  // compute-thread index
    // order (nullable): the slice of each workgroup, in dispatch order
    const uint32_t slice = order ? order[blockIdx.x] : xcd_slice(blockIdx.x, gridDim.x);
    OpArgs A;
    A.C = C;
    A.ldz = (size_t)ld;
    A.nwords = nwords;
    static_assert(LW == 1 || SAT, "two-word lanes in saturating launches only");
    constexpr uint32_t SL = SW / LW;  // lanes per op
    A.sld = (nwords + 1u) & ~1u;
    A.w = slice * SW + LW * (ctid % SL);
    A.wok = !loader && A.w < nwords;
    A.vw = A.wok ? min((uint32_t)LW, nwords - A.w) : 0u;
    A.grp = ctid / SL;
    A.ngrp = (blockDim.x - kLoaderThreads) / SL;
    A.sink = scratch + (size_t)blockIdx.x * kRoworSinkWords + LW * tid;
    A.rows = rows;
    A.sat = satbits;
    A.sbase = sbase;
    A.sbits = sbits;
    A.loaded = A.stored = 0;
    A.lead = (ctid % SL) == 0;
    {
        const uint32_t tail = n & 63u;
        const uint64_t last = tail ? (1ull << tail) - 1ull : ~0ull;
        A.fullw = !A.wok ? 0ull : (A.w + 1 < nwords ? ~0ull : last);
        A.fullw1 = !A.wok || A.w + 1 >= nwords ? 0ull : (A.w + 2 < nwords ? ~0ull : last);
        A.gmask = (SL == 64 ? ~0ull : ((1ull << SL) - 1ull)) << ((tid & 63u) / SL * SL);
    }
    // Once every real row is full in this slice, all later ops are full
    // results into full rows: the workgroup stops.  A slice with a single
    // valid column starts with that column's identity row full.
    //
    // persist (streamed builds, one chunk of the stream per launch): per
    // slice {done, full-row count, real-row bits}, carried from the launch
    // of the previous chunk; a slice already done returns at once.  Scratch
    // rows never outlive a time step, so their bits start at zero.
    //
    // ZERO keeps a second bitmap of rows that are all zero in the slice: at
    // the start every real row except those of the slice's own nodes (the
    // identity), minus the rows an earlier chunk made non-zero (persisted
    // complemented, so that a cleared state means a fresh identity).
    // Scratch rows start unknown.
    const uint32_t c0 = slice * SW * 64u;
    const bool single = c0 + 1 == n;
    const uint32_t rwords = sbase / 32;  // words of real-row bits
    const uint32_t swords = (sbits + 31) / 32;
    // persisted per slice: done, full count, full bits, non-zero bits (all
    // ones, i.e. unknown, after a launch without ZERO)
    const size_t pslice = 2 * (size_t)rwords + 2;
    uint32_t *pst = (SAT && CHUNK) ? persist + (size_t)slice * pslice : nullptr;
    uint32_t *zbits = satbits + swords;
    int32_t nfull = single ? 1 : 0;
    int32_t nzero = 0;
    if (SAT) {
        if (pst) {
            if (pst[0]) return;
            nfull = (int32_t)pst[1];
            if (single && !((pst[2 + (c0 >> 5)] >> (c0 & 31u)) & 1u)) ++nfull;
        }
        if (ZERO && tid == 0) zcount0 = 0;
        __syncthreads();
        const uint32_t c1 = min(n, c0 + SW * 64u);  // the slice's own nodes: [c0, c1)
        for (uint32_t i = tid; i < swords; i += blockDim.x) {
            uint32_t v = (pst && i < rwords) ? pst[2 + i] : 0u;
            if (single && i == (c0 >> 5)) v |= 1u << (c0 & 31u);
            satbits[i] = v;
            if (ZERO) {
                uint32_t z = 0u;
                if (i < rwords) {
                    const uint32_t r0 = 32 * i;
                    // rows < n, minus the identity rows, minus persisted non-zero rows
                    z = r0 + 32 <= n ? ~0u : (r0 < n ? (1u << (n - r0)) - 1u : 0u);
                    const uint32_t a = max(r0, c0), b = min(r0 + 32, c1);
                    if (a < b) {
                        const uint32_t len = b - a;
                        z &= ~((len == 32 ? ~0u : ((1u << len) - 1u)) << (a - r0));
                    }
                    if (pst) z &= ~pst[2 + rwords + i];
                    if (z) atomicAdd(&zcount0, (int32_t)__popc(z));
                }
                zbits[i] = z;
            }
        }
        if (tid < 3) {
            fdelta[tid] = 0;
            zdelta[tid] = 0;
        }
        if (ZERO) {
            __syncthreads();
            nzero = zcount0;
        }
    }
    A.nfull = fdelta;
    A.dfull = A.dzero = 0;
    A.zb = zbits;
    A.nzero = zdelta;
    A.zon = false;
    const bool stopped = level_loop<SW, UC, SAT, MAX8, ZERO, LW>(
        A, s, n, loader, tid, ctid, frame, fcount, worklist, fdelta, zdelta, nfull, nzero);
    if (loader) return;
    count_add(traffic, A.loaded);
    count_add(traffic + 1, A.stored);
    if (pst) {
        for (uint32_t i = ctid; i < rwords; i += blockDim.x - kLoaderThreads) {
            pst[2 + i] = satbits[i];
            pst[2 + rwords + i] = ZERO ? ~zbits[i] : ~0u;
        }
        if (ctid == 0) {
            pst[1] = (uint32_t)nfull;
            if (nfull == (int32_t)n) {
                pst[0] = 1u;
                atomicAdd(done_count, 1u);
            }
        }
    }
}

// The plain recurrence with level-to-level forwarding (forwarded op form,
// tn_internal.h).  Each op's result r also goes into this level's LDS
// result frame, at the op's index; an operand that the level just before
// wrote is read from there instead of memory, and a row that the next level
// overwrites is not stored.  About half of all row reads and stores of an
// activity-driven stream leave memory this way: almost every op reads one
// row the level before wrote, and that row is rewritten right away.
//
// Cold operands (rows last written two or more levels before) do not
// depend on the level just before, so their loads are issued one level
// early: right after the barrier that starts level l, the compute waves
// issue the cold loads of level l + 1, then run level l on the values that
// arrived meanwhile.  A load of level l + 1 reads a row stored at level
// l - 1 or earlier, by a store issued before that barrier: the workgroup's
// waves share one CU and its in-order vector memory path, so the load sees
// it (the barrier itself does not wait for memory operations, which keeps
// the loads in flight across it).  Loader waves keep a ring of three op
// frames (the level run, the level whose cold loads are in flight, the
// level being loaded); results alternate between two LDS frames.
constexpr uint32_t kFwdFrames = 3;

// The lane group's index, opaque to the optimizer: the op indices derived
// from it are then formed where they are used instead of being hoisted out
// of the level loop into registers of their own (one per op slot).
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}

template <int UC, int LW>
struct ColdVals {
    typename LaneT<LW>::T x[UC], y[UC];
};

// The cold operands of the level in `frame` (forwarded ones are not read).
template <int SW, int UC, bool OFF32, int LW>
__device__ __forceinline__ void fwd_issue(OpArgs &A, const op4 *frame, uint32_t cnt,
                                          ColdVals<UC, LW> &c) {
    using T = typename LaneT<LW>::T;
    constexpr uint32_t NG = (1024 - kLoaderThreads) / (SW / LW);
    const uint32_t g = opaque(A.grp);
#pragma unroll
    for (int k = 0; k < UC; ++k) {
        const uint32_t j = g + k * NG;
        const op4 o = frame[min(j, kOpsLevelCap - 1)];
        const bool v = j < cnt;
        const bool hx = o.x & kFwdHot, hy = o.y & kFwdHot;
        // only the lanes that need a row read it: a lane sent to a sink
        // instead costs the CU's texture units as much as a real access
        if (v && !hx && A.wok) c.x[k] = *(const T *)fwd_addr<OFF32>(A, o.x, true);
        if (v && !hy && A.wok) c.y[k] = *(const T *)fwd_addr<OFF32>(A, o.y, true);
        A.loaded += ((v && !hx) ? A.vw : 0u) + ((v && !hy) ? A.vw : 0u);
    }
}

// Runs the level in `frame` with its cold values in c.  keep clears a
// lane's word past the row's last one (LW = 2), so padding stays zero.
template <int SW, int UC, bool OFF32, int LW>
__device__ __forceinline__ void fwd_apply(OpArgs &A, const op4 *frame, uint32_t cnt,
                                          const ColdVals<UC, LW> &c, const uint64_t *res_prev,
                                          uint64_t *res_cur, uint32_t lig,
                                          typename LaneT<LW>::T keep) {
    using T = typename LaneT<LW>::T;
    constexpr uint32_t SL = SW / LW;  // lanes per op
    constexpr uint32_t NG = (1024 - kLoaderThreads) / SL;
    const T *rp = reinterpret_cast<const T *>(res_prev);
    T *rc = reinterpret_cast<T *>(res_cur);
    const uint32_t g = opaque(A.grp);
#pragma unroll
    for (int k = 0; k < UC; ++k) {
        const uint32_t j = g + k * NG;
        const op4 o = frame[min(j, kOpsLevelCap - 1)];
        const bool v = j < cnt;
        // a cold operand's low bits are a row id: its (unused) read is
        // clamped into the frame
        const T lx = rp[min(o.x & kFwdSlotMask, kFwdLevelCap) * SL + lig];
        const T ly = rp[min(o.y & kFwdSlotMask, kFwdLevelCap) * SL + lig];
        const T r = (((o.x & kFwdHot) ? lx : c.x[k]) | ((o.y & kFwdHot) ? ly : c.y[k])) & keep;
        // slot kFwdLevelCap takes the writes of lanes with no op
        rc[(v ? j : kFwdLevelCap) * SL + lig] = r;
        // kNoRow has the no-store bit too: it is never stored
        const bool s1 = v && !(o.z & kFwdNoStore);
        const bool s2 = v && !(o.w & kFwdNoStore);
        if (s1 && A.wok) *(T *)fwd_addr<OFF32>(A, o.z, true) = r;
        if (s2 && A.wok) *(T *)fwd_addr<OFF32>(A, o.w, true) = r;
        A.stored += (s1 ? A.vw : 0u) + (s2 ? A.vw : 0u);
    }
}

// The level loop of k_rowor_fwd over the levels of the forwarded schedule
// s, on loader and compute waves (A set up by the caller; results: two
// result frames of kFwdLevelCap + 1 slots of SW words).  Loader waves return
// after their loop, compute waves after the last level's stores are issued.
template <int SW, int UC, bool OFF32, int LW>
__device__ __forceinline__ void fwd_loop(OpArgs &A, const DevOps &s, bool loader, uint32_t tid,
                                         uint32_t ctid, op4 (*frame)[kOpsLevelCap],
                                         uint32_t *fcount, uint64_t *results) {
    constexpr uint32_t kFrameWords = (kFwdLevelCap + 1) * SW;
    const uint32_t L = s.L;
    if (loader) {
        // levels 0 and 1 before the first barrier; at the barrier that
        // starts level l, frame (l + 2) % 3 receives level l + 2.  Starts
        // and ops are fetched a level ahead into registers (hA, hB; the
        // loop is unrolled by two so that they never change registers).
        put_level(frame[0], fetch_ops(s, level_start(s, 0), tid), tid);
        put_level(frame[1], fetch_ops(s, level_start(s, 1), tid), tid);
        if (tid == 0) {
            fcount[0] = level_start(s, 1) - level_start(s, 0);
            fcount[1] = level_start(s, 2) - level_start(s, 1);
        }
        uint32_t p2 = level_start(s, 2), p3 = level_start(s, 3);
        HeldOps hA = fetch_ops(s, p2, tid);
        uint32_t p4 = level_start(s, 4);
        HeldOps hB = fetch_ops(s, p3, tid);
        // at level l: h holds the ops of level l + 2, p2..p4 the starts of
        // levels l + 2 .. l + 4
        auto feed = [&](uint32_t l, HeldOps &h) {
            __syncthreads();
            const uint32_t nf = (l + 2) % kFwdFrames;
            put_level(frame[nf], h, tid);
            if (tid == 0) fcount[nf] = p3 - p2;
            const uint32_t q = p4;
            p2 = p3;
            p3 = q;
            p4 = level_start(s, l + 5);
            h = fetch_ops(s, q, tid);
        };
        for (uint32_t l = 0; l < L; l += 2) {
            feed(l, hA);
            if (l + 1 >= L) break;
            feed(l + 1, hB);
        }
        return;
    }
    constexpr uint32_t SL = SW / LW;
    const uint32_t lig = ctid % SL;
    typename LaneT<LW>::T keep;
    if constexpr (LW == 1) {
        keep = ~0ull;
    } else {
        keep = u64x2{~0ull, A.w + 1 < A.nwords ? ~0ull : 0ull};
    }
    ColdVals<UC, LW> cA, cB;
    // Runs level l with cur holding its cold values, after issuing level
    // l + 1's into nxt.  The issue runs on every path (a level past the last
    // has no ops and issues nothing) and level 0's own issue comes before
    // the loop, so the code between a load and its use is the same on every
    // path: the compiler's wait before the use then leaves the loads issued
    // after it in flight (a join with a path that skipped the issue would
    // make it wait for those too).  Within an issue, each load is masked to
    // the lanes whose operand is cold: 109 -> 83 ms for the plain
    // recurrence at n = 10^5, m = 10^7, where every lane had read a row or
    // its sink.
    auto period = [&](uint32_t l, ColdVals<UC, LW> &cur, ColdVals<UC, LW> &nxt) {
        __syncthreads();
        const uint32_t nf = (l + 1) % kFwdFrames;
        fwd_issue<SW, UC, OFF32, LW>(A, frame[nf], fcount[nf], nxt);
        const uint32_t cf = l % kFwdFrames;
        fwd_apply<SW, UC, OFF32, LW>(A, frame[cf], fcount[cf], cur,
                                     results + (size_t)((l + 1) & 1u) * kFrameWords,
                                     results + (size_t)(l & 1u) * kFrameWords, lig, keep);
    };
    // level 0's cold values (frame 0 is written before the loaders' first
    // barrier, which the first period waits at)
    __syncthreads();
    fwd_issue<SW, UC, OFF32, LW>(A, frame[0], fcount[0], cA);
    {
        fwd_issue<SW, UC, OFF32, LW>(A, frame[1], fcount[1], cB);
        fwd_apply<SW, UC, OFF32, LW>(A, frame[0], fcount[0], cA, results + kFrameWords, results,
                                     lig, keep);
    }
    for (uint32_t l = 1; l < L; l += 2) {
        period(l, cB, cA);
        if (l + 1 >= L) break;
        period(l + 1, cA, cB);
    }
}

// LW words per lane: SW / LW lanes per op (LW = 2 needs even ld and a
// 16-byte aligned matrix).
template <int SW, int UC, bool OFF32, int LW>
__global__ void __launch_bounds__(1024)
k_rowor_fwd(uint64_t *__restrict__ C, int64_t ld, uint32_t nwords, DevOps s,
            uint64_t *__restrict__ scratch, uint64_t *__restrict__ rows,
            unsigned long long *__restrict__ traffic) {
    static_assert(((1024 - kLoaderThreads) / (SW / LW)) * UC >= kFwdLevelCap, "a level per pass");
    constexpr uint32_t SL = SW / LW;
    __shared__ op4 frame[kFwdFrames][kOpsLevelCap];
    __shared__ uint32_t fcount[kFwdFrames];
    // dynamic: two result frames of kFwdLevelCap + 1 slots (the last one a
    // sink) of SW words
    extern __shared__ __attribute__((aligned(16))) uint64_t results[];
    if (s.L == 0 || s.nops == 0) return;
    const uint32_t tid = threadIdx.x;
    const bool loader = tid < kLoaderThreads;
    const uint32_t ctid = tid - kLoaderThreads;
    const uint32_t slice = xcd_slice(blockIdx.x, gridDim.x);
    OpArgs A;
    A.C = C;
    A.ldz = (size_t)ld;
    A.nwords = nwords;
    A.sld = (nwords + 1u) & ~1u;
    A.w = slice * SW + LW * (ctid % SL);
    A.wok = !loader && A.w < nwords;
    A.vw = A.wok ? min((uint32_t)LW, nwords - A.w) : 0u;
    A.grp = ctid / SL;
    A.ngrp = (blockDim.x - kLoaderThreads) / SL;
    A.sink = scratch + (size_t)blockIdx.x * kRoworSinkWords + LW * tid;
    A.rows = rows;
    A.loaded = A.stored = 0;
    A.ld32 = (uint32_t)ld;
    fwd_loop<SW, UC, OFF32, LW>(A, s, loader, tid, ctid, frame, fcount, results);
    if (loader) return;
    count_add(traffic, A.loaded);
    count_add(traffic + 1, A.stored);
}

// The same recurrence on 16-word slices (whole 128-byte lines of a row):
// two result frames of 769 x 128 bytes would not fit in LDS beside the op
// frames, so one frame serves both levels.  A level reads its forwarded
// operands from the frame, stores its results to memory, waits at a second
// barrier (LDS only: the next level's cold loads stay in flight) until
// every wave has read the frame, then writes its results into it.  Cold
// values are held for y of every op and for x of the first UCX ops per lane
// group only (the schedule puts the ops with both operands from memory
// first; about 1 % of an activity-driven stream's ops).  A lane whose op
// past those has x from memory too (levels right after the identity)
// loads it on the spot and waits for all its loads.  At n = 10^5 its 98
// workgroups take 174 ms for the plain recurrence where 196 of 8 words
// take 121 ms; it is the kernel of slice_words = 16.
template <int UC, int UCX>
struct ColdY {
    uint64_t y[UC], x[UCX];
};

template <int SW, int UC, int UCX, bool OFF32>
__device__ __forceinline__ void fwd1_issue(OpArgs &A, const op4 *frame, uint32_t cnt,
                                           ColdY<UC, UCX> &c) {
    constexpr uint32_t NG = (1024 - kLoaderThreads) / SW;
    const uint32_t g = opaque(A.grp);
#pragma unroll
    for (int k = 0; k < UC; ++k) {
        const uint32_t j = g + k * NG;
        const op4 o = frame[min(j, kOpsLevelCap - 1)];
        const bool v = j < cnt;
        const bool hy = o.y & kFwdHot;
        if (v && !hy && A.wok) c.y[k] = *fwd_addr<OFF32>(A, o.y, true);
        A.loaded += (v && A.wok && !hy) ? 1u : 0u;
        if (k < UCX) {
            const bool hx = o.x & kFwdHot;
            if (v && !hx && A.wok) c.x[k] = *fwd_addr<OFF32>(A, o.x, true);
            A.loaded += (v && A.wok && !hx) ? 1u : 0u;
        }
    }
}

// Waits for this wave's LDS accesses, then for every wave of the workgroup;
// memory operations in flight stay in flight.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int SW, int UC, int UCX, bool OFF32>
__device__ __forceinline__ void fwd1_apply(OpArgs &A, const op4 *frame, uint32_t cnt,
                                           const ColdY<UC, UCX> &c, uint64_t *res,
                                           uint32_t lig) {
    constexpr uint32_t NG = (1024 - kLoaderThreads) / SW;
    uint64_t r[UC];
    const uint32_t g = opaque(A.grp);
#pragma unroll
    for (int k = 0; k < UC; ++k) {
        const uint32_t j = g + k * NG;
        const op4 o = frame[min(j, kOpsLevelCap - 1)];
        const bool v = j < cnt;
        const uint64_t lx = res[min(o.x & kFwdSlotMask, kFwdLevelCap) * SW + lig];
        const uint64_t ly = res[min(o.y & kFwdSlotMask, kFwdLevelCap) * SW + lig];
        uint64_t x = (o.x & kFwdHot) ? lx : (k < UCX ? c.x[k < UCX ? k : 0] : 0ull);
        if (k >= UCX && v && !(o.x & kFwdHot)) {
            x = *fwd_addr<OFF32>(A, o.x, true);
            // vmcnt(0) (expcnt and lgkmcnt left at their maxima): the wait
            // pass then knows the value has landed
            __builtin_amdgcn_s_waitcnt(0x0F70);
            A.loaded += A.wok ? 1u : 0u;
        }
        r[k] = x | ((o.y & kFwdHot) ? ly : c.y[k]);
        const bool s1 = v && !(o.z & kFwdNoStore);
        const bool s2 = v && !(o.w & kFwdNoStore);
        if (s1 && A.wok) *fwd_addr<OFF32>(A, o.z, true) = r[k];
        if (s2 && A.wok) *fwd_addr<OFF32>(A, o.w, true) = r[k];
        A.stored += ((s1 && A.wok) ? 1u : 0u) + ((s2 && A.wok) ? 1u : 0u);
    }
    lds_barrier();
    const uint32_t g2 = opaque(A.grp);
#pragma unroll
    for (int k = 0; k < UC; ++k) {
        const uint32_t j = g2 + k * NG;
        res[(j < cnt ? j : kFwdLevelCap) * SW + lig] = r[k];
    }
}

template <int SW, int UC, int UCX, bool OFF32>
__global__ void __launch_bounds__(1024)
k_rowor_fwd1(uint64_t *__restrict__ C, int64_t ld, uint32_t nwords, DevOps s,
             uint64_t *__restrict__ scratch, uint64_t *__restrict__ rows,
             unsigned long long *__restrict__ traffic) {
    static_assert(((1024 - kLoaderThreads) / SW) * UC >= kFwdLevelCap, "a level per pass");
    __shared__ op4 frame[kFwdFrames][kOpsLevelCap];
    __shared__ uint32_t fcount[kFwdFrames];
    // dynamic: one result frame of kFwdLevelCap + 1 slots (the last one a
    // sink) of SW words
    extern __shared__ uint64_t results[];
    const uint32_t L = s.L;
    if (L == 0 || s.nops == 0) return;
    const uint32_t tid = threadIdx.x;
    const bool loader = tid < kLoaderThreads;
    const uint32_t ctid = tid - kLoaderThreads;
    const uint32_t slice = xcd_slice(blockIdx.x, gridDim.x);
    OpArgs A;
    A.C = C;
    A.ldz = (size_t)ld;
    A.nwords = nwords;
    A.sld = (nwords + 1u) & ~1u;
    A.w = slice * SW + (ctid % SW);
    A.wok = !loader && A.w < nwords;
    A.grp = ctid / SW;
    A.ngrp = (blockDim.x - kLoaderThreads) / SW;
    A.sink = scratch + (size_t)blockIdx.x * kRoworSinkWords + tid;
    A.rows = rows;
    A.loaded = A.stored = 0;
    A.ld32 = (uint32_t)ld;
    if (loader) {
        // as in k_rowor_fwd, with the second barrier of every level
        put_level(frame[0], fetch_ops(s, level_start(s, 0), tid), tid);
        put_level(frame[1], fetch_ops(s, level_start(s, 1), tid), tid);
        if (tid == 0) {
            fcount[0] = level_start(s, 1) - level_start(s, 0);
            fcount[1] = level_start(s, 2) - level_start(s, 1);
        }
        uint32_t p2 = level_start(s, 2), p3 = level_start(s, 3);
        HeldOps hA = fetch_ops(s, p2, tid);
        uint32_t p4 = level_start(s, 4);
        HeldOps hB = fetch_ops(s, p3, tid);
        auto feed = [&](uint32_t l, HeldOps &h) {
            __syncthreads();
            const uint32_t nf = (l + 2) % kFwdFrames;
            put_level(frame[nf], h, tid);
            if (tid == 0) fcount[nf] = p3 - p2;
            const uint32_t q = p4;
            p2 = p3;
            p3 = q;
            p4 = level_start(s, l + 5);
            h = fetch_ops(s, q, tid);
            lds_barrier();
        };
        for (uint32_t l = 0; l < L; l += 2) {
            feed(l, hA);
            if (l + 1 >= L) break;
            feed(l + 1, hB);
        }
        return;
    }
    const uint32_t lig = ctid % SW;
    ColdY<UC, UCX> cA, cB;
    // as in k_rowor_fwd: level 0 peeled, every issue unconditional
    auto period = [&](uint32_t l, ColdY<UC, UCX> &cur, ColdY<UC, UCX> &nxt) {
        __syncthreads();
        const uint32_t nf = (l + 1) % kFwdFrames;
        fwd1_issue<SW, UC, UCX, OFF32>(A, frame[nf], fcount[nf], nxt);
        const uint32_t cf = l % kFwdFrames;
        fwd1_apply<SW, UC, UCX, OFF32>(A, frame[cf], fcount[cf], cur, results, lig);
    };
    __syncthreads();
    fwd1_issue<SW, UC, UCX, OFF32>(A, frame[0], fcount[0], cA);
    fwd1_issue<SW, UC, UCX, OFF32>(A, frame[1], fcount[1], cB);
    fwd1_apply<SW, UC, UCX, OFF32>(A, frame[0], fcount[0], cA, results, lig);
    for (uint32_t l = 1; l < L; l += 2) {
        period(l, cB, cA);
        if (l + 1 >= L) break;
        period(l + 1, cA, cB);
    }
    count_add(traffic, A.loaded);
    count_add(traffic + 1, A.stored);
}

// The per-slice state of the saturating kernel (launch_rowor_global's
// persist) rebuilt from the matrix itself: for slice s, bit r of its full
// row bits is set iff row r holds every column of the slice, and its count
// is the number of such rows.  One wavefront per 64 rows of a span of RW
// words (RW / SW slices; at least 8 words, so that narrow slices still read
// 64-byte row segments), neighbouring wavefronts on the neighbouring spans
// of the same rows (a row's words are contiguous): groups of RW lanes read
// one row segment each, RW rows per lane with every load issued before the
// first compare; the SW lanes of a slice AND their checks, lane r of the
// wave collects row r's result for each slice of the span, and one ballot
// per slice gives two bitmap words.  The state must be zero before
// (launch_fill_u32).
template <int SW, int RW>
__global__ void __launch_bounds__(256)
k_slice_full_state(const uint64_t *__restrict__ C, int64_t ld, uint32_t n, uint32_t nwords,
                   uint32_t slices, uint32_t *__restrict__ persist) {
    static_assert(RW % SW == 0 && RW <= 64, "a span holds whole slices");
    constexpr uint32_t G = 64 / RW;  // rows per load instruction
    constexpr uint32_t S = RW / SW;  // slices per span
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t g = lane / RW, j = lane % RW;
    const uint32_t rwords = ((n + 31u) & ~31u) / 32;
    const size_t pslice = 2 * (size_t)rwords + 2;
    const uint32_t blocks = (n + 63) / 64;
    const uint32_t tail = n & 63u;
    const uint64_t last = tail ? (1ull << tail) - 1ull : ~0ull;
    const uint32_t spans = (slices + S - 1) / S;
    const size_t jobs = (size_t)spans * blocks;
    for (size_t job = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; job < jobs;
         job += ((size_t)gridDim.x * blockDim.x) >> 6) {
        const uint32_t span = (uint32_t)(job % spans);
        const uint32_t rb = (uint32_t)(job / spans);
        const uint32_t r0 = rb * 64;
        const uint32_t w = span * RW + j;
        const bool wok = w < nwords;  // words past the last one check as full
        const uint64_t want = w + 1 == nwords ? last : ~0ull;
        uint64_t v[RW];
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const uint32_t r = r0 + k * G + g;
            v[k] = (wok && r < n) ? C[(size_t)r * (size_t)ld + w] : want;
        }
        bool mine[S];
#pragma unroll
        for (int q = 0; q < (int)S; ++q) mine[q] = false;
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            int f = (r0 + k * G + g < n && v[k] == want) ? 1 : 0;
#pragma unroll
            for (uint32_t off = 1; off < SW; off <<= 1) f &= __shfl_xor(f, off);
            // row r0 + lane is row k * G + g of iteration k = lane / G
#pragma unroll
            for (int q = 0; q < (int)S; ++q) {
                const int t = __shfl(f, (int)((lane % G) * RW + q * SW));
                if (lane / G == (uint32_t)k) mine[q] = t != 0;
            }
        }
        const uint32_t word = rb * 2;
#pragma unroll
        for (int q = 0; q < (int)S; ++q) {
            const uint32_t slice = span * S + q;
            const uint64_t b = __ballot(mine[q]);
            if (slice >= slices) break;
            uint32_t *pst = persist + (size_t)slice * pslice;
            if (lane == 0 && word < rwords) pst[2 + word] = (uint32_t)b;
            if (lane == 1 && word + 1 < rwords) pst[2 + word + 1] = (uint32_t)(b >> 32);
            if (lane == 0 && b) atomicAdd(pst + 1, (uint32_t)__popcll(b));
        }
    }
}

// The order in which a saturating launch takes its slices: by the count of
// full real rows in the slice state, fewest first, ties by slice index, so
// the slices with the most work left start first and the lightest fill the
// compute units that free up.  One thread per slice counts the slices that
// come before it (a strict total order, so the ranks are a permutation).
__global__ void __launch_bounds__(256)
k_slice_order(const uint32_t *__restrict__ persist, uint32_t pslice, uint32_t slices,
              uint32_t *__restrict__ order) {
    __shared__ uint32_t key[256];
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const uint32_t mine = s < slices ? persist[(size_t)s * pslice + 1] : 0u;
    uint32_t rank = 0;
    for (uint32_t j0 = 0; j0 < slices; j0 += 256u) {
        const uint32_t j = j0 + threadIdx.x;
        __syncthreads();
        key[threadIdx.x] = j < slices ? persist[(size_t)j * pslice + 1] : 0u;
        __syncthreads();
        const uint32_t m = min(256u, slices - j0);
        for (uint32_t k = 0; k < m; ++k) {
            const uint32_t c = key[k];
            rank += (c < mine || (c == mine && j0 + k < s)) ? 1u : 0u;
        }
    }
    if (s < slices) order[rank] = s;
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t *__restrict__ p, uint32_t n, int32_t v) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Whether word column w lies in a slice that a saturating launch left all
// ones in every row (its done word in the slice state; no state: none).
__device__ __forceinline__ bool word_done(const uint32_t *persist, uint32_t pslice, uint32_t sw,
                                          uint32_t w) {
    return persist && persist[(size_t)(w / sw) * pslice] != 0u;
}

// out[u] = popcount of row u: one wavefront per row, lanes stride the words.
// With a slice state (persist: pslice words per slice of sw words), a word
// of a slice left all ones counts its valid columns without a read.
__global__ void __launch_bounds__(256)
k_out_sizes(const uint64_t *__restrict__ C, uint32_t n, int64_t ld, uint32_t nwords,
            int32_t *__restrict__ out, const uint32_t *__restrict__ persist, uint32_t pslice,
            uint32_t sw) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwave = (gridDim.x * blockDim.x) >> 6;
    // this lane's done words: their columns once, a row read for the rest
    int base = 0;
    bool any_open = false;
    for (uint32_t j = lane; j < nwords; j += 64) {
        if (word_done(persist, pslice, sw, j))
            base += (j + 1 < nwords || (n & 63u) == 0) ? 64 : (int)(n & 63u);
        else
            any_open = true;
    }
    if (__ballot(any_open) == 0) {
        // every word of the row is done: the same count for every row,
        // reduced once (a shuffle step is an LDS permute)
        int total = base;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off, 64);
        for (uint32_t r = wave * 64 + lane; r < n; r += nwave * 64) out[r] = total;
        return;
    }
    for (uint32_t r = wave; r < n; r += nwave) {
        const uint64_t *row = C + (size_t)r * (size_t)ld;
        int c = base;
        if (any_open) {
            for (uint32_t j = lane; j < nwords; j += 64)
                if (!word_done(persist, pslice, sw, j)) c += __popcll(row[j]);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
        if (lane == 0) out[r] = c;
    }
}

// in[w] = number of rows with bit w: each lane owns one word column over a
// share of a chunk of rows and adds the words into 16 bit-planes (a
// bit-sliced ripple counter, 64 column counters at once).  The four waves of
// a workgroup take quarters of the chunk, add their 64 counts per lane into
// LDS, and the workgroup adds each column's total to in[] once: one global
// atomic per column and chunk of kInRowsPerChunk rows.
constexpr uint32_t kInRowsPerChunk = 4096;  // per wave 1024 < 2^16: 16 planes suffice
// With a slice state, a word column of a slice left all ones has n in
// every column: the first chunk adds it, no chunk reads the column.
__global__ void __launch_bounds__(256)
k_in_sizes(const uint64_t *__restrict__ C, uint32_t n, int64_t ld, uint32_t nwords,
           int32_t *__restrict__ in, const uint32_t *__restrict__ persist, uint32_t pslice,
           uint32_t sw) {
    __shared__ int32_t cnt[64 * 64];  // [bit][column word]: a wave's lanes on distinct banks
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (uint32_t i = threadIdx.x; i < 64 * 64; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const uint32_t j = blockIdx.x * 64 + lane;
    const uint32_t share = kInRowsPerChunk / 4;
    const uint32_t r0 = blockIdx.y * kInRowsPerChunk + wave * share;
    const uint32_t r1 = min(n, r0 + share);
    const bool done = j < nwords && word_done(persist, pslice, sw, j);
    if (done && blockIdx.y == 0 && wave == 0) {
        const uint32_t bits = (j + 1 < nwords || (n & 63u) == 0) ? 64u : (n & 63u);
        for (uint32_t b = 0; b < bits; ++b) atomicAdd(&cnt[b * 64 + lane], (int32_t)n);
    }
    if (j < nwords && r0 < r1 && !done) {
        uint64_t c[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) c[i] = 0;
        const uint64_t *col = C + j;
        uint32_t r = r0;
        for (; r + 8 <= r1; r += 8) {
            uint64_t x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = col[(size_t)(r + q) * (size_t)ld];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                uint64_t carry = x[q];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const uint64_t t = c[i] & carry;
                    c[i] ^= carry;
                    carry = t;
                }
            }
        }
        for (; r < r1; ++r) {
            uint64_t carry = col[(size_t)r * (size_t)ld];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint64_t t = c[i] & carry;
                c[i] ^= carry;
                carry = t;
            }
        }
        for (uint32_t b = 0; b < 64; ++b) {
            int32_t v = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) v |= (int32_t)((c[i] >> b) & 1ull) << i;
            if (v) atomicAdd(&cnt[b * 64 + lane], v);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
        const uint32_t node = blockIdx.x * 64 * 64 + i;  // (column word) * 64 + bit
        const int32_t v = cnt[(i & 63u) * 64 + (i >> 6)];
        if (node < n && v) atomicAdd(in + node, v);
    }
}

template <int SW, int UC>
hipError_t rowor_variant(const DevOps &s, uint32_t n, uint64_t *C, int64_t ld, uint64_t *scratch,
                         uint64_t *rows, uint32_t scratch_rows, unsigned long long *traffic,
                         bool saturation, uint32_t *persist, unsigned int *done_count,
                         uint32_t zero_levels, const uint32_t *order, hipStream_t st) {
    const uint32_t nwords = (n + 63) / 64;
    const uint32_t slices = (nwords + SW - 1) / SW;
    const uint32_t sbase = (n + 31u) & ~31u;
    const uint64_t sbits = (uint64_t)sbase + scratch_rows + 1;
    const size_t lds = (size_t)((sbits + 31) / 32) * 4;
    // two words per lane where every matrix row starts on 16 bytes (scratch
    // rows always do: scratch_stride)
    constexpr int LW2 = (SW >= 2 && SW <= 16) ? 2 : 1;
    const bool two = LW2 == 2 && ld % 2 == 0 && ((uintptr_t)C & 15u) == 0;
    if (saturation && lds <= kRoworSatLds) {
        DevOps rest = s;
        // zero phase: the first levels, while most row slices are still all
        // zero, in a launch of its own that also keeps the zero bitmap; the
        // slice state carries over to the launch of the remaining levels,
        // which keeps only the full-row bits (the zero phase's per-level work
        // would cost more than it saves there)
        if (zero_levels > 0 && persist && 2 * lds <= kRoworSatLds) {
            DevOps head = s;
            head.L = min(zero_levels, s.L);
            auto kz = two ? k_rowor_global<SW, UC, true, true, false, true, LW2>
                          : k_rowor_global<SW, UC, true, true, false, true, 1>;
            hipError_t e = hipFuncSetAttribute((const void *)kz,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)(2 * lds));
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kz, dim3(slices), dim3(1024), 2 * lds, st, C, ld, n, nwords, head,
                               scratch, rows, sbase, (uint32_t)sbits, traffic, persist, done_count,
                               (const uint32_t *)nullptr);
            e = hipGetLastError();
            if (e != hipSuccess || head.L == s.L) return e;
            rest.L = s.L - head.L;
            rest.lvl = s.lvl + head.L;
        }
        auto k = persist ? (two ? k_rowor_global<SW, UC, true, true, false, false, LW2>
                                : k_rowor_global<SW, UC, true, true, false, false, 1>)
                         : (two ? k_rowor_global<SW, UC, true, false, false, false, LW2>
                                : k_rowor_global<SW, UC, true, false, false, false, 1>);
        hipError_t e = hipFuncSetAttribute((const void *)k,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(slices), dim3(1024), lds, st, C, ld, n, nwords, rest, scratch,
                           rows, sbase, (uint32_t)sbits, traffic, persist, done_count, order);
    } else {
        hipLaunchKernelGGL((k_rowor_global<SW, UC, false, false>), dim3(slices), dim3(1024), 0,
                           st, C, ld, n, nwords, s, scratch, rows, 0u, 1u, traffic,
                           (uint32_t *)nullptr, (unsigned int *)nullptr, order);
    }
    return hipGetLastError();
}

}  // namespace

// Register rows are short (2^b bytes), so the level loop is bound by the
// instructions each lane issues per level, not by bytes: one word per lane
// (two for rows past 32 words) measured fastest (2x over 8 words at 256
// registers), one workgroup per word column.
static uint32_t rowmax_slice_words(uint32_t nwords) { return nwords <= 32 ? 1u : 2u; }

hipError_t launch_rowmax_global(const DevOps &s, uint32_t rows, uint32_t nwords, uint64_t *M,
                                int64_t ld, uint64_t *scratch, uint32_t scratch_rows,
                                unsigned long long *traffic, hipStream_t st) {
    (void)scratch_rows;
    if (s.L == 0) return hipSuccess;
    const uint32_t sw = rowmax_slice_words(nwords);
    const uint32_t slices = (nwords + sw - 1) / sw;
    uint64_t *mrows = scratch + (size_t)slices * kRoworSinkWords;
    switch (sw) {
        case 1:
            hipLaunchKernelGGL((k_rowor_global<1, 2, false, false, true>), dim3(slices), dim3(1024),
                               0, st, M, ld, rows, nwords, s, scratch, mrows, 0u, 1u,
                               traffic, (uint32_t *)nullptr, (unsigned int *)nullptr,
                               (const uint32_t *)nullptr);
            break;
        case 2:
            hipLaunchKernelGGL((k_rowor_global<2, 3, false, false, true>), dim3(slices), dim3(1024),
                               0, st, M, ld, rows, nwords, s, scratch, mrows, 0u, 1u,
                               traffic, (uint32_t *)nullptr, (unsigned int *)nullptr,
                               (const uint32_t *)nullptr);
            break;
        case 4:
            hipLaunchKernelGGL((k_rowor_global<4, 5, false, false, true>), dim3(slices), dim3(1024),
                               0, st, M, ld, rows, nwords, s, scratch, mrows, 0u, 1u,
                               traffic, (uint32_t *)nullptr, (unsigned int *)nullptr,
                               (const uint32_t *)nullptr);
            break;
        case 8:
            hipLaunchKernelGGL((k_rowor_global<8, 10, false, false, true>), dim3(slices),
                               dim3(1024), 0, st, M, ld, rows, nwords, s, scratch, mrows, 0u, 1u,
                               traffic, (uint32_t *)nullptr, (unsigned int *)nullptr,
                               (const uint32_t *)nullptr);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

uint32_t rowmax_workgroups(uint32_t nwords) {
    const uint32_t sw = rowmax_slice_words(nwords);
    return (nwords + sw - 1) / sw;
}

uint32_t default_slice_words(uint32_t n, int64_t ld) {
    (void)ld;
    const uint32_t nwords = (n + 63) / 64;
    // at least ~256 workgroups when the matrix is wide enough, else narrow
    // slices; 16 words = one 128-byte line per row access
    if (nwords >= 16 * 256) return 16;
    if (nwords >= 8 * 192) return 8;
    if (nwords >= 4 * 128) return 4;
    if (nwords >= 2 * 64) return 2;
    return 1;
}

hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t v, hipStream_t st) {
    if (count == 0) return hipSuccess;
    if (count > 0xffffffffull) return hipErrorInvalidValue;
    uint32_t blocks = (uint32_t)((count + 255) / 256);
    if (blocks > 4096u) blocks = 4096u;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, st, (int32_t *)p, (uint32_t)count,
                       (int32_t)v);
    return hipGetLastError();
}

hipError_t launch_identity(uint64_t *C, uint32_t n, int64_t ld, unsigned long long *traffic,
                           hipStream_t st) {
    const uint32_t blocks = n < 65536u ? n : 65536u;
    hipLaunchKernelGGL(k_identity, dim3(blocks), dim3(256), 0, st, C, n, ld, traffic);
    return hipGetLastError();
}

uint32_t rowor_workgroups(uint32_t n, uint32_t slice_words) {
    const uint32_t nwords = (n + 63) / 64;
    return (nwords + slice_words - 1) / slice_words;
}

hipError_t launch_rowor_global(const DevOps &s, uint32_t n, uint64_t *C, int64_t ld,
                               uint32_t slice_words, uint64_t *scratch, uint32_t sink_slots,
                               uint32_t scratch_rows, unsigned long long *traffic,
                               bool saturation, uint32_t *persist, unsigned int *done_count,
                               uint32_t zero_levels, const uint32_t *order, hipStream_t st) {
    if (s.L == 0) return hipSuccess;
    if (slice_words == 0 || sink_slots < rowor_workgroups(n, slice_words)) return hipErrorInvalidValue;
    uint64_t *rows = scratch + (size_t)sink_slots * kRoworSinkWords;
    switch (slice_words) {
        // UC: ops per lane group and level, so that (896 / SW) * UC >= 1024
        case 1: return rowor_variant<1, 2>(s, n, C, ld, scratch, rows, scratch_rows, traffic, saturation, persist, done_count, zero_levels, order, st);
        case 2: return rowor_variant<2, 3>(s, n, C, ld, scratch, rows, scratch_rows, traffic, saturation, persist, done_count, zero_levels, order, st);
        case 4: return rowor_variant<4, 5>(s, n, C, ld, scratch, rows, scratch_rows, traffic, saturation, persist, done_count, zero_levels, order, st);
        case 8: return rowor_variant<8, 10>(s, n, C, ld, scratch, rows, scratch_rows, traffic, saturation, persist, done_count, zero_levels, order, st);
        case 16: return rowor_variant<16, 8>(s, n, C, ld, scratch, rows, scratch_rows, traffic, saturation, persist, done_count, zero_levels, order, st);
        case 32: return rowor_variant<32, 8>(s, n, C, ld, scratch, rows, scratch_rows, traffic, saturation, persist, done_count, zero_levels, order, st);
        case 64: return rowor_variant<64, 8>(s, n, C, ld, scratch, rows, scratch_rows, traffic, saturation, persist, done_count, zero_levels, order, st);
        default: return hipErrorInvalidValue;
    }
}

template <int SW, int UC, int LW>
hipError_t rowor_fwd_variant(const DevOps &s, uint32_t n, uint64_t *C, int64_t ld,
                             uint64_t *scratch, uint64_t *rows, bool off32,
                             unsigned long long *traffic, hipStream_t st) {
    const uint32_t nwords = (n + 63) / 64;
    const uint32_t slices = (nwords + SW - 1) / SW;
    const size_t lds = sizeof(uint64_t) * 2 * (kFwdLevelCap + 1) * SW;
    auto k = off32 ? k_rowor_fwd<SW, UC, true, LW> : k_rowor_fwd<SW, UC, false, LW>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(slices), dim3(1024), lds, st, C, ld, nwords, s, scratch, rows,
                       traffic);
    return hipGetLastError();
}

template <int SW, int UC, int UCX>
hipError_t rowor_fwd1_variant(const DevOps &s, uint32_t n, uint64_t *C, int64_t ld,
                              uint64_t *scratch, uint64_t *rows, bool off32,
                              unsigned long long *traffic, hipStream_t st) {
    const uint32_t nwords = (n + 63) / 64;
    const uint32_t slices = (nwords + SW - 1) / SW;
    const size_t lds = sizeof(uint64_t) * (kFwdLevelCap + 1) * SW;
    auto k = off32 ? k_rowor_fwd1<SW, UC, UCX, true> : k_rowor_fwd1<SW, UC, UCX, false>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(slices), dim3(1024), lds, st, C, ld, nwords, s, scratch, rows,
                       traffic);
    return hipGetLastError();
}

bool rowor_fwd_supported(uint32_t n, uint32_t slice_words) {
    return slice_words <= 16 && n < (1u << 30);
}

// Row offsets (row * stride + word) of the matrix and of the scratch rows
// fit 32 bits, with rows and strides below 2^24 (fwd_addr).
static bool rowor_fwd_off32(uint32_t n, int64_t ld, uint32_t scratch_rows) {
    const uint64_t nwords = (n + 63) / 64;
    return n < (1u << 24) && ld < (1 << 24) && scratch_rows + 1 < (1u << 24) &&
           (uint64_t)n * (uint64_t)ld < (1ull << 32) &&
           (uint64_t)(scratch_rows + 1) * scratch_stride((uint32_t)nwords) < (1ull << 32);
}

hipError_t launch_rowor_fwd(const DevOps &s, uint32_t n, uint64_t *C, int64_t ld,
                            uint32_t slice_words, uint64_t *scratch, uint32_t sink_slots,
                            uint32_t scratch_rows, unsigned long long *traffic, hipStream_t st) {
    if (s.L == 0) return hipSuccess;
    if (!rowor_fwd_supported(n, slice_words) || slice_words == 0 ||
        sink_slots < rowor_workgroups(n, slice_words))
        return hipErrorInvalidValue;
    uint64_t *rows = scratch + (size_t)sink_slots * kRoworSinkWords;
    const bool o32 = rowor_fwd_off32(n, ld, scratch_rows);
    // two words per lane where every row starts on 16 bytes (scratch rows
    // always do: scratch_stride)
    const bool two = ld % 2 == 0 && ((uintptr_t)C & 15u) == 0;
    switch (slice_words) {
        // UC: ops per lane group, so that (896 / (SW / LW)) * UC >= kFwdLevelCap
        case 1: return rowor_fwd_variant<1, 1, 1>(s, n, C, ld, scratch, rows, o32, traffic, st);
        case 2:
            return two ? rowor_fwd_variant<2, 1, 2>(s, n, C, ld, scratch, rows, o32, traffic, st)
                       : rowor_fwd_variant<2, 2, 1>(s, n, C, ld, scratch, rows, o32, traffic, st);
        case 4:
            return two ? rowor_fwd_variant<4, 2, 2>(s, n, C, ld, scratch, rows, o32, traffic, st)
                       : rowor_fwd_variant<4, 4, 1>(s, n, C, ld, scratch, rows, o32, traffic, st);
        case 8:
            return two ? rowor_fwd_variant<8, 4, 2>(s, n, C, ld, scratch, rows, o32, traffic, st)
                       : rowor_fwd_variant<8, 7, 1>(s, n, C, ld, scratch, rows, o32, traffic, st);
        case 16: return rowor_fwd1_variant<16, 14, 2>(s, n, C, ld, scratch, rows, o32, traffic, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_slice_full_state(const uint64_t *C, int64_t ld, uint32_t n,
                                   uint32_t slice_words, uint32_t *persist, hipStream_t st) {
    const uint32_t nwords = (n + 63) / 64;
    const uint32_t slices = rowor_workgroups(n, slice_words);
    hipError_t e = launch_fill_u32(persist, rowor_persist_words(n, slice_words), 0u, st);
    if (e != hipSuccess) return e;
    // spans of at least 8 words
    const uint32_t span_words = slice_words < 8 ? 8 : slice_words;
    const size_t spans = ((size_t)nwords + span_words - 1) / span_words;
    const size_t waves = spans * ((n + 63) / 64);
    const uint32_t blocks = (uint32_t)std::min<size_t>((waves + 3) / 4, 65536);
    switch (slice_words) {
        case 1: hipLaunchKernelGGL((k_slice_full_state<1, 8>), dim3(blocks), dim3(256), 0, st, C, ld, n, nwords, slices, persist); break;
        case 2: hipLaunchKernelGGL((k_slice_full_state<2, 8>), dim3(blocks), dim3(256), 0, st, C, ld, n, nwords, slices, persist); break;
        case 4: hipLaunchKernelGGL((k_slice_full_state<4, 8>), dim3(blocks), dim3(256), 0, st, C, ld, n, nwords, slices, persist); break;
        case 8: hipLaunchKernelGGL((k_slice_full_state<8, 8>), dim3(blocks), dim3(256), 0, st, C, ld, n, nwords, slices, persist); break;
        case 16: hipLaunchKernelGGL((k_slice_full_state<16, 16>), dim3(blocks), dim3(256), 0, st, C, ld, n, nwords, slices, persist); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_slice_order(const uint32_t *persist, uint32_t n, uint32_t slice_words,
                              uint32_t *order, hipStream_t st) {
    if (slice_words == 0) return hipErrorInvalidValue;
    const uint32_t slices = rowor_workgroups(n, slice_words);
    const size_t pslice = rowor_persist_words(n, slice_words) / slices;
    if (slices == 0) return hipSuccess;
    hipLaunchKernelGGL(k_slice_order, dim3((slices + 255) / 256), dim3(256), 0, st, persist,
                       (uint32_t)pslice, slices, order);
    return hipGetLastError();
}

uint32_t tail_slice_words(uint32_t n, uint32_t slice_words, int num_cus) {
    uint32_t sw = slice_words;
    const uint32_t cap = 4u * (uint32_t)(num_cus > 0 ? num_cus : 1);
    while (sw > 1 && rowor_workgroups(n, sw / 2) <= cap) sw /= 2;
    return sw;
}

hipError_t launch_out_sizes(const uint64_t *C, uint32_t n, int64_t ld, int32_t *out_sizes,
                            hipStream_t st, const uint32_t *persist, uint32_t state_sw) {
    const uint32_t nwords = (n + 63) / 64;
    uint32_t blocks = (n + 3) / 4;
    if (blocks > 16384u) blocks = 16384u;
    // with a state every wave first reads the done words of its lanes: fewer
    // waves, each taking more rows
    if (persist && blocks > 2048u) blocks = 2048u;
    const uint32_t pslice = persist ? (uint32_t)(2 * (((size_t)n + 31) / 32) + 2) : 0u;
    hipLaunchKernelGGL(k_out_sizes, dim3(blocks), dim3(256), 0, st, C, n, ld, nwords, out_sizes,
                       persist, pslice, state_sw ? state_sw : 1u);
    return hipGetLastError();
}

hipError_t launch_in_sizes(const uint64_t *C, uint32_t n, int64_t ld, int32_t *in_sizes,
                           hipStream_t st, const uint32_t *persist, uint32_t state_sw) {
    const uint32_t nwords = (n + 63) / 64;
    uint32_t fb = (n + 255) / 256;
    if (fb > 4096u) fb = 4096u;
    hipLaunchKernelGGL(k_fill_i32, dim3(fb), dim3(256), 0, st, in_sizes, n, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((nwords + 63) / 64, (n + kInRowsPerChunk - 1) / kInRowsPerChunk);
    const uint32_t pslice = persist ? (uint32_t)(2 * (((size_t)n + 31) / 32) + 2) : 0u;
    hipLaunchKernelGGL(k_in_sizes, grid, dim3(256), 0, st, C, n, ld, nwords, in_sizes, persist,
                       pslice, state_sw ? state_sw : 1u);
    return hipGetLastError();
}

}  // namespace tn
