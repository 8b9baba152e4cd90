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

#include "tn_internal.h"

namespace tn {

namespace {

// Workgroups are dispatched round-robin over the 8 XCDs of the chip; map the
// workgroup index so that each XCD receives a contiguous range of slices
// (adjacent slices share cache lines of the same rows).
__device__ __forceinline__ uint32_t xcd_slice(uint32_t b, uint32_t nb) {
    const uint32_t x = b & 7u, k = b >> 3;
    const uint32_t q = nb >> 3, r = nb & 7u;
    return x * q + min(x, r) + k;
}

__global__ void __launch_bounds__(256) k_identity(uint64_t *__restrict__ C, uint32_t n, int64_t ld) {
    for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
        uint64_t *row = C + (size_t)r * (size_t)ld;
        const int64_t diag = (int64_t)(r >> 6);
        const uint64_t bit = 1ull << (r & 63u);
        for (int64_t j = threadIdx.x; j < ld; j += blockDim.x) row[j] = (j == diag) ? bit : 0ull;
    }
}

// One workgroup per slice of SW word columns; SW consecutive lanes update the
// SW words of one item's rows, so each row access is one contiguous
// 8*SW-byte segment.  Per level, a lane group holds up to U pair items (and
// UG compound-item gathers) in registers and issues all their row loads before
// any store.  The level boundaries are staged in LDS a window ahead and the
// items of the next level are loaded while the current level runs, so a level
// costs one round trip for its rows plus the store acknowledgement its
// closing barrier waits for.  A level with compound items keeps the gathered
// rows in registers across one extra barrier (read all, then write all).
constexpr uint32_t kLevelWindow = 512;

template <int U>
__device__ __forceinline__ void load_items(uint2 (&it)[U], const uint2 *__restrict__ pairs,
                                           uint32_t first, uint32_t end, uint32_t ngrp) {
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const uint32_t idx = first + k * ngrp;
        it[k] = (idx < end) ? pairs[idx] : make_uint2(0xffffffffu, 0u);
    }
}

template <int U>
__device__ __forceinline__ void load_rows(const uint64_t *__restrict__ C, size_t ldz, uint32_t w,
                                          bool wok, const uint2 (&it)[U], uint64_t (&a)[U],
                                          uint64_t (&b)[U]) {
#pragma unroll
    for (int k = 0; k < U; ++k) {
        if (it[k].x != 0xffffffffu && wok) {
            a[k] = C[(size_t)it[k].x * ldz + w];
            b[k] = C[(size_t)(it[k].y & kNodeMask) * ldz + w];
        }
    }
}

template <int U>
__device__ __forceinline__ void store_rows(uint64_t *__restrict__ C, size_t ldz, uint32_t w, bool wok,
                                           const uint2 (&it)[U], const uint64_t (&a)[U],
                                           const uint64_t (&b)[U]) {
#pragma unroll
    for (int k = 0; k < U; ++k) {
        if (it[k].x != 0xffffffffu && wok) {
            const uint64_t r = a[k] | b[k];
            C[(size_t)it[k].x * ldz + w] = r;
            if (!(it[k].y & kDirBit)) C[(size_t)(it[k].y & kNodeMask) * ldz + w] = r;
        }
    }
}

__device__ __forceinline__ uint64_t gather_row(const uint64_t *__restrict__ C, size_t ldz, uint32_t w,
                                               const DevSchedule &s, uint32_t gi) {
    uint64_t acc = 0;
    const uint32_t s0 = s.gat_ptr[gi], s1 = s.gat_ptr[gi + 1];
    for (uint32_t q = s0; q < s1; ++q) acc |= C[(size_t)s.gat_src[q] * ldz + w];
    return acc;
}

template <int SW, int U, int UG>
__global__ void __launch_bounds__(1024)
k_rowor_global(uint64_t *__restrict__ C, int64_t ld, uint32_t nwords, DevSchedule s,
               uint64_t *__restrict__ scratch) {
    __shared__ uint32_t win_p[2][kLevelWindow];
    __shared__ uint32_t win_g[2][kLevelWindow];
    const uint32_t slice = xcd_slice(blockIdx.x, gridDim.x);
    const uint32_t w = slice * SW + (threadIdx.x % SW);
    const bool wok = w < nwords;
    const uint32_t grp = threadIdx.x / SW;
    const uint32_t ngrp = blockDim.x / SW;
    const uint32_t chunk = ngrp * U;
    const size_t ldz = (size_t)ld;
    const uint32_t L = s.L;
    // level boundaries of window 0 and 1 (entries past L repeat entry L)
    for (uint32_t i = threadIdx.x; i < 2 * kLevelWindow; i += blockDim.x) {
        const uint32_t l = min(i, L);
        win_p[i / kLevelWindow][i % kLevelWindow] = s.lvl_pair[l];
        win_g[i / kLevelWindow][i % kLevelWindow] = s.lvl_gat[l];
    }
    __syncthreads();
    auto lp = [&](uint32_t l) { return win_p[(l / kLevelWindow) & 1u][l % kLevelWindow]; };
    auto lg = [&](uint32_t l) { return win_g[(l / kLevelWindow) & 1u][l % kLevelWindow]; };
    uint32_t p0 = lp(0), p1 = lp(1);
    uint32_t g0 = lg(0);
    uint2 cur[U];
    load_items<U>(cur, s.pairs, p0 + grp, p1, ngrp);
    for (uint32_t l = 0; l < L; ++l) {
        if (l % kLevelWindow == 0 && l > 0) {
            // refill the buffer of the window before this one with the window
            // after it; it was last read three levels ago, before a barrier
            const uint32_t nb = l / kLevelWindow + 1;
            for (uint32_t i = threadIdx.x; i < kLevelWindow; i += blockDim.x) {
                const uint32_t ll = min(nb * kLevelWindow + i, L);
                win_p[nb & 1u][i] = s.lvl_pair[ll];
                win_g[nb & 1u][i] = s.lvl_gat[ll];
            }
        }
        const uint32_t p2 = lp(min(l + 2, L));
        const uint32_t g1 = lg(l + 1);
        uint2 nxt[U];
        load_items<U>(nxt, s.pairs, p1 + grp, p2, ngrp);
        uint64_t a[U], b[U];
        load_rows<U>(C, ldz, w, wok, cur, a, b);
        const uint32_t ng = g1 - g0;
        uint64_t gacc[UG];
        if (ng > 0 && ng <= ngrp * UG) {
#pragma unroll
            for (int k = 0; k < UG; ++k) {
                const uint32_t gi = g0 + grp + k * ngrp;
                if (gi < g1 && wok) gacc[k] = gather_row(C, ldz, w, s, gi);
            }
        }
        store_rows<U>(C, ldz, w, wok, cur, a, b);
        // levels wider than one register chunk
        for (uint32_t base = p0 + chunk + grp; base < p1; base += chunk) {
            uint2 more[U];
            load_items<U>(more, s.pairs, base, p1, ngrp);
            load_rows<U>(C, ldz, w, wok, more, a, b);
            store_rows<U>(C, ldz, w, wok, more, a, b);
        }
        if (ng > 0) {
            if (ng <= ngrp * UG) {
                __syncthreads();
#pragma unroll
                for (int k = 0; k < UG; ++k) {
                    const uint32_t gi = g0 + grp + k * ngrp;
                    if (gi < g1 && wok) C[(size_t)s.gat_tgt[gi] * ldz + w] = gacc[k];
                }
            } else {
                // more gathers than register slots: stage through scratch rows
                for (uint32_t gi = g0 + grp; gi < g1; gi += ngrp)
                    if (wok) scratch[(size_t)(gi - g0) * nwords + w] = gather_row(C, ldz, w, s, gi);
                __syncthreads();
                for (uint32_t gi = g0 + grp; gi < g1; gi += ngrp)
                    if (wok) C[(size_t)s.gat_tgt[gi] * ldz + w] = scratch[(size_t)(gi - g0) * nwords + w];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < U; ++k) cur[k] = nxt[k];
        p0 = p1;
        p1 = p2;
        g0 = g1;
    }
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t *__restrict__ p, uint32_t n, int32_t v) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// out[u] = popcount of row u: one wavefront per row, lanes stride the words.
__global__ void __launch_bounds__(256)
k_out_sizes(const uint64_t *__restrict__ C, uint32_t n, int64_t ld, uint32_t nwords,
            int32_t *__restrict__ out) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwave = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t r = wave; r < n; r += nwave) {
        const uint64_t *row = C + (size_t)r * (size_t)ld;
        int c = 0;
        for (uint32_t j = lane; j < nwords; j += 64) c += __popcll(row[j]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
        if (lane == 0) out[r] = c;
    }
}

// in[w] = number of rows with bit w: each lane owns one word column over a
// chunk of rows and adds the words into 16 bit-planes (a bit-sliced ripple
// counter, 64 column counters at once), then adds the 64 counts to in[].
constexpr uint32_t kInRowsPerChunk = 2048;  // < 2^16: 16 planes suffice
__global__ void __launch_bounds__(64)
k_in_sizes(const uint64_t *__restrict__ C, uint32_t n, int64_t ld, uint32_t nwords,
           int32_t *__restrict__ in) {
    const uint32_t j = blockIdx.x * 64 + threadIdx.x;
    if (j >= nwords) return;
    const uint32_t r0 = blockIdx.y * kInRowsPerChunk;
    const uint32_t r1 = min(n, r0 + kInRowsPerChunk);
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
        const uint32_t node = 64 * j + b;
        if (node >= n) break;
        int32_t cnt = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) cnt |= (int32_t)((c[i] >> b) & 1ull) << i;
        if (cnt) atomicAdd(in + node, cnt);
    }
}

template <int SW, int U, int UG = 1>
hipError_t rowor_variant(const DevSchedule &s, uint64_t *C, int64_t ld, uint32_t nwords,
                         uint64_t *scratch, hipStream_t st) {
    const uint32_t slices = (nwords + SW - 1) / SW;
    hipLaunchKernelGGL((k_rowor_global<SW, U, UG>), dim3(slices), dim3(1024), 0, st, C, ld, nwords, s,
                       scratch);
    return hipGetLastError();
}

}  // namespace

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

hipError_t launch_identity(uint64_t *C, uint32_t n, int64_t ld, hipStream_t st) {
    const uint32_t blocks = n < 65536u ? n : 65536u;
    hipLaunchKernelGGL(k_identity, dim3(blocks), dim3(256), 0, st, C, n, ld);
    return hipGetLastError();
}

hipError_t launch_rowor_global(const DevSchedule &s, uint64_t *C, int64_t ld, uint32_t slice_words,
                               uint64_t *scratch, hipStream_t st) {
    const uint32_t nwords = (s.n + 63) / 64;
    if (s.L == 0) return hipSuccess;
    switch (slice_words) {
        case 1: return rowor_variant<1, 2>(s, C, ld, nwords, scratch, st);
        case 2: return rowor_variant<2, 2>(s, C, ld, nwords, scratch, st);
        case 4: return rowor_variant<4, 4>(s, C, ld, nwords, scratch, st);
        case 8: return rowor_variant<8, 8>(s, C, ld, nwords, scratch, st);
        case 16: return rowor_variant<16, 8>(s, C, ld, nwords, scratch, st);
        case 32: return rowor_variant<32, 8>(s, C, ld, nwords, scratch, st);
        case 64: return rowor_variant<64, 8>(s, C, ld, nwords, scratch, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_out_sizes(const uint64_t *C, uint32_t n, int64_t ld, int32_t *out_sizes,
                            hipStream_t st) {
    const uint32_t nwords = (n + 63) / 64;
    uint32_t blocks = (n + 3) / 4;
    if (blocks > 16384u) blocks = 16384u;
    hipLaunchKernelGGL(k_out_sizes, dim3(blocks), dim3(256), 0, st, C, n, ld, nwords, out_sizes);
    return hipGetLastError();
}

hipError_t launch_in_sizes(const uint64_t *C, uint32_t n, int64_t ld, int32_t *in_sizes,
                           hipStream_t st) {
    const uint32_t nwords = (n + 63) / 64;
    uint32_t fb = (n + 255) / 256;
    if (fb > 4096u) fb = 4096u;
    hipLaunchKernelGGL(k_fill_i32, dim3(fb), dim3(256), 0, st, in_sizes, n, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((nwords + 63) / 64, (n + kInRowsPerChunk - 1) / kInRowsPerChunk);
    hipLaunchKernelGGL(k_in_sizes, grid, dim3(64), 0, st, C, n, ld, nwords, in_sizes);
    return hipGetLastError();
}

}  // namespace tn
