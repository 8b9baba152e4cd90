// Network hashing (Sec. 4.1) and fusion of the hashed proxies (Sec. 4.2).
//
// Hash: h_j(u) = (acc_0(x0) ^ acc_1(x1) ^ acc_2(x2)) mod K, where x0 / x1 are
// the low / high 32 bits of u, x2 = x0 + x1, and acc_i folds the coefficients
// of row i of table A_j with (x * acc + a) mod (2^61 - 1).  The product is
// formed exactly in 128 bits and reduced with 2^61 = 1 (mod 2^61 - 1).
//
// Fusion: the estimated out-component of u keeps node w iff bit h_j(w) of row
// h_j(u) of every proxy P_j is set.  For a chunk q of 64 nodes w and a hash
// j, the lifted table Lt[q][j][r] packs those 64 bits for every super-node
// r; it is the transpose of the 64 proxy columns h_j(w), so it is built from
// the transposed proxies with 64 x 64 bit transposes inside a wavefront.  The
// estimate of u is then sum_q popcount(AND_j Lt[q][j][h_j(u)]), evaluated
// with the tables of a chunk staged in LDS.
#include <hip/hip_runtime.h>

#include "tn_device.h"
#include "tn_hash.h"

namespace tn {

namespace {

constexpr uint64_t kP61 = (1ull << 61) - 1;

// (x * acc + a) mod (2^61 - 1), x < 2^34, acc < 2^61, a < 2^61 - 1.
__device__ __forceinline__ uint64_t mult_add_mod(uint64_t x, uint64_t acc, uint64_t a) {
    uint64_t lo = x * acc;
    uint64_t hi = __umul64hi(x, acc);
    const uint64_t lo2 = lo + a;
    hi += (lo2 < lo) ? 1ull : 0ull;
    lo = lo2;
    // value = hi * 2^64 + lo;  2^64 = 8 (mod p), 2^61 = 1 (mod p)
    uint64_t r = (lo & kP61) + (lo >> 61) + (hi << 3);
    r = (r & kP61) + (r >> 61);
    return r >= kP61 ? r - kP61 : r;
}

__device__ __forceinline__ uint64_t poly(const uint64_t *__restrict__ Ai, int order, uint64_t x) {
    uint64_t acc = Ai[0] % kP61;
    for (int l = 1; l < order; ++l) acc = mult_add_mod(x, acc, Ai[l]);
    return acc;
}

__global__ void __launch_bounds__(256)
k_hash_buckets(uint32_t n, uint32_t H, const uint64_t *__restrict__ coeffs, int order, uint32_t K,
               uint32_t *__restrict__ bucket) {
    const size_t total = (size_t)n * H;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t j = (uint32_t)(i / n);
        const uint64_t u = i - (size_t)j * n;
        const uint64_t *A = coeffs + (size_t)j * 3 * order;
        const uint64_t x0 = u & 0xffffffffull, x1 = u >> 32, x2 = x0 + x1;
        const uint64_t h = poly(A, order, x0) ^ poly(A + order, order, x1) ^
                           poly(A + 2 * order, order, x2);
        bucket[i] = (uint32_t)(h % K);
    }
}

__global__ void __launch_bounds__(256) k_zero_i32(int32_t *__restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void __launch_bounds__(256)
k_bucket_counts(uint32_t n, uint32_t H, uint32_t K, const uint32_t *__restrict__ bucket,
                int32_t *__restrict__ count) {
    const size_t total = (size_t)n * H;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t j = (uint32_t)(i / n);
        atomicAdd(count + (size_t)j * K + bucket[i], 1);
    }
}

// Transposes the 64 x 64 bit block held one row per lane (bit b of lane i's
// word is entry (i, b)); afterwards lane b holds column b.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t masks[6] = {0x00000000ffffffffull, 0x0000ffff0000ffffull,
                               0x00ff00ff00ff00ffull, 0x0f0f0f0f0f0f0f0full,
                               0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const uint32_t s = 32u >> k;
        const uint64_t y = (uint64_t)__shfl_xor((unsigned long long)x, (int)s, 64);
        if (lane & s) {
            const uint64_t t = ((y >> s) ^ x) & masks[k];
            x ^= t;
        } else {
            const uint64_t t = ((x >> s) ^ y) & masks[k];
            x ^= t << s;
        }
    }
    return x;
}

// PT_j = transpose of P_j (K x K bits): one wavefront per run of kLiftRun
// 64 x 64 blocks along a row block; lane i reads kLiftRun consecutive words
// of row 64 br + i (the loads after the first hit the sector the first
// brought in), then each block is transposed and written.
constexpr uint32_t kLiftRun = 8;
__global__ void __launch_bounds__(256)
k_transpose_proxies(uint32_t H, uint32_t K, int64_t ldK, const uint64_t *__restrict__ P,
                    uint64_t *__restrict__ PT) {
    const uint32_t kw = (K + 63) / 64;
    const uint32_t runs = (kw + kLiftRun - 1) / kLiftRun;
    const size_t jobs = (size_t)H * kw * runs;
    const uint32_t lane = threadIdx.x & 63u;
    for (size_t job = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; job < jobs;
         job += ((size_t)gridDim.x * blockDim.x) >> 6) {
        const uint32_t j = (uint32_t)(job / ((size_t)kw * runs));
        const uint32_t rem = (uint32_t)(job - (size_t)j * kw * runs);
        const uint32_t br = rem / runs, bc0 = rem % runs * kLiftRun;  // row block, first word block
        const uint64_t *Pj = P + (size_t)j * K * ldK;
        const uint32_t r = br * 64 + lane;
        uint64_t x[kLiftRun];
#pragma unroll
        for (uint32_t t = 0; t < kLiftRun; ++t)
            x[t] = (r < K && bc0 + t < kw) ? Pj[(size_t)r * ldK + bc0 + t] : 0ull;
#pragma unroll
        for (uint32_t t = 0; t < kLiftRun; ++t) {
            if (bc0 + t >= kw) break;  // uniform: the whole wave
            const uint64_t y = wave_transpose64(x[t]);  // lane b: bits r of column 64 (bc0 + t) + b
            const uint32_t c = (bc0 + t) * 64 + lane;
            if (c < K) PT[(size_t)j * K * ldK + (size_t)c * ldK + br] = y;
        }
    }
}

// bsum[j][wd] = sum of count[j][c] over the 64 super-nodes c of word wd
// (those below K): one wavefront per (j, wd).
__global__ void __launch_bounds__(256)
k_block_sums(uint32_t H, uint32_t K, const int32_t *__restrict__ count, int32_t *__restrict__ bsum) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t kw = (K + 63) / 64;
    const size_t blocks = (size_t)H * kw;
    for (size_t b = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; b < blocks;
         b += ((size_t)gridDim.x * blockDim.x) >> 6) {
        const uint32_t j = (uint32_t)(b / kw), c = (uint32_t)(b % kw) * 64 + lane;
        int32_t v = c < K ? count[(size_t)j * K + c] : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) bsum[b] = v;
    }
}

// One pass over every proxy row r of P_j, one wavefront per row, its lanes
// on consecutive words: full[j][r] = 1 iff the row has all K bits set, and
// (rowsum not NULL) rowsum[j][r] = sum of count[j][c] over the super-nodes
// c set in the row.  A full word adds its block sum, an empty one nothing,
// and each other word one count load per lane (lane l: super-node 64 wd + l).
__global__ void __launch_bounds__(256)
k_row_sums_full(uint32_t H, uint32_t K, int64_t ldK, const uint64_t *__restrict__ P,
                const int32_t *__restrict__ count, const int32_t *__restrict__ bsum,
                int32_t *__restrict__ rowsum, uint8_t *__restrict__ full) {
    const uint32_t lane = threadIdx.x & 63u;
    const size_t rows = (size_t)H * K;
    const uint32_t kw = (K + 63) / 64;
    const uint64_t last = (K % 64) ? ((1ull << (K % 64)) - 1ull) : ~0ull;
    for (size_t row = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; row < rows;
         row += ((size_t)gridDim.x * blockDim.x) >> 6) {
        const uint32_t j = (uint32_t)(row / K);
        const uint64_t *Pr = P + (size_t)j * K * ldK + (row - (size_t)j * K) * ldK;
        const int32_t *cj = count + (size_t)j * K;
        int32_t acc = 0;
        bool all = true;
        for (uint32_t wd0 = 0; wd0 < kw; wd0 += 64) {
            const uint32_t wd = wd0 + lane;
            const uint64_t word = wd < kw ? Pr[wd] : 0ull;
            const bool fullw = wd < kw && word == (wd + 1 == kw ? last : ~0ull);
            all &= wd >= kw || fullw;
            if (!rowsum) continue;
            if (fullw) acc += bsum[(size_t)j * kw + wd];
            // the other non-empty words, one at a time over the wavefront
            uint64_t partial = __ballot(wd < kw && word != 0ull && !fullw);
            while (partial) {
                const uint32_t p = (uint32_t)__builtin_ctzll(partial);
                partial &= partial - 1ull;
                const uint64_t wp =
                    ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(word >> 32), (int)p) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)word, (int)p);
                const uint32_t c = (wd0 + p) * 64 + lane;
                if (c < K && ((wp >> lane) & 1ull)) acc += cj[c];
            }
        }
        const bool row_full = __ballot(!all) == 0ull;
        if (rowsum) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        }
        if (lane == 0) {
            if (rowsum) rowsum[row] = acc;
            full[row] = row_full ? 1 : 0;
        }
    }
}

__global__ void __launch_bounds__(256)
k_lifted_sizes(uint32_t n, uint32_t H, const uint32_t *__restrict__ bucket,
               const int32_t *__restrict__ rowsum, uint32_t K, int32_t *__restrict__ lifted) {
    const size_t total = (size_t)n * H;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t j = (uint32_t)(i / n);
        lifted[i] = rowsum[(size_t)j * K + bucket[i]];
    }
}

// Lt[(q - q0) * H * K + j * K + r], bit i = P_j[r][h_j(64 q + i)] (0 past n):
// one wavefront per (q, j, run of kLiftRun 64-row blocks); lane i gathers
// words br of the transposed proxy row h_j(64 q + i) for the run's blocks
// (consecutive words of one row, so the loads after the first hit the
// sector it brought in), then each block is transposed and written.
__global__ void __launch_bounds__(256)
k_build_lifted(uint32_t n, uint32_t H, uint32_t K, int64_t ldK, const uint64_t *__restrict__ PT,
               const uint32_t *__restrict__ bucket, uint32_t q0, uint32_t nq,
               uint64_t *__restrict__ Lt) {
    const uint32_t kw = (K + 63) / 64;
    const uint32_t runs = (kw + kLiftRun - 1) / kLiftRun;
    const size_t jobs = (size_t)nq * H * runs;
    const uint32_t lane = threadIdx.x & 63u;
    for (size_t job = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; job < jobs;
         job += ((size_t)gridDim.x * blockDim.x) >> 6) {
        const uint32_t br0 = (uint32_t)(job % runs) * kLiftRun;
        const uint32_t j = (uint32_t)((job / runs) % H);
        const uint32_t qq = (uint32_t)(job / ((size_t)runs * H));
        const uint64_t w = (uint64_t)(q0 + qq) * 64 + lane;
        uint64_t x[kLiftRun];
        const uint64_t *row = nullptr;
        if (w < n) row = PT + (size_t)j * K * ldK + (size_t)bucket[(size_t)j * n + w] * ldK;
#pragma unroll
        for (uint32_t t = 0; t < kLiftRun; ++t)
            x[t] = (row && br0 + t < kw) ? row[br0 + t] : 0ull;
#pragma unroll
        for (uint32_t t = 0; t < kLiftRun; ++t) {
            if (br0 + t >= kw) break;  // uniform: the whole wave
            const uint64_t y = wave_transpose64(x[t]);
            const uint32_t r = (br0 + t) * 64 + lane;
            if (r < K) Lt[((size_t)qq * H + j) * K + r] = y;
        }
    }
}

// A node whose proxy row is full in every hash keeps every node: est = n.
// Every other node is appended to `list` for the AND/popcount kernel.
__global__ void __launch_bounds__(256)
k_split_full(uint32_t n, uint32_t H, uint32_t K, const uint32_t *__restrict__ bucket,
             const uint8_t *__restrict__ full, int32_t *__restrict__ est,
             uint32_t *__restrict__ list, uint32_t *__restrict__ count) {
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        bool all = true;
        for (uint32_t j = 0; j < H && all; ++j) all = full[(size_t)j * K + bucket[(size_t)j * n + u]] != 0;
        if (all) {
            est[u] = (int32_t)n;
        } else {
            est[u] = 0;
            list[atomicAdd(count, 1u)] = u;
        }
    }
}

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

// Tables of g hashes of one chunk (g K words at src) into LDS at dst,
// straight from memory with no registers: a wave's 64 lanes fill 64 units
// from the wave's LDS base, lane l at l units; 16-byte units where the
// tables start on 16 bytes (K even), else 4-byte ones.  Completes at the
// next barrier (which waits for the wave's own transfers).
__device__ __forceinline__ void stage_tables(const uint64_t *src, uint32_t words, uint32_t K,
                                             uint64_t *dst) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t waves = blockDim.x >> 6;
    if (K % 2 == 0) {
        const uint32_t units = words / 2;
        for (uint32_t c0 = wave * 64; c0 < units; c0 += waves * 64)
            if (c0 + lane < units)
                __builtin_amdgcn_global_load_lds((glb_void *)(src + 2 * (size_t)(c0 + lane)),
                                                 (lds_void *)(dst + 2 * (size_t)c0), 16, 0, 0);
    } else {
        const uint32_t units = words * 2;
        const uint32_t *s32 = (const uint32_t *)src;
        uint32_t *d32 = (uint32_t *)dst;
        for (uint32_t c0 = wave * 64; c0 < units; c0 += waves * 64)
            if (c0 + lane < units)
                __builtin_amdgcn_global_load_lds((glb_void *)(s32 + c0 + lane),
                                                 (lds_void *)(d32 + c0), 4, 0, 0);
    }
}

// est[u] += sum over the chunks q of this launch of popcount(AND_j Lt[q][j][h_j(u)]).
// A workgroup owns kUPT nodes u per thread (a node block) and one of the
// launch's ranges of `per` chunks; the counts of the ranges add up in est
// (integer atomics, so the order does not matter).  Every node block stages
// the same tables, so the workgroups of one chunk range are numbered
// consecutively and given to one XCD (xcd_slice): they run there together
// and read the tables through that XCD's L2 rather than each from HBM.  With
// LDS,
// the tables of G hashes of one chunk are staged in LDS at a time (K words
// each), else (tables too large for LDS) they are read where they are, in
// L2; the AND of a chunk is carried in registers across the hash groups.
constexpr int kUPT = 8;
constexpr int kQB = 2;
constexpr uint32_t kRecombineThreads = 1024;
constexpr size_t kRecombineLds = 160 * 1024;  // LDS of one CU
template <bool LDS>
__global__ void __launch_bounds__(kRecombineThreads)
k_recombine_est(uint32_t n, uint32_t H, uint32_t K, uint32_t G, const uint32_t *__restrict__ bucket,
                const uint64_t *__restrict__ Lt, uint32_t q_first, uint32_t q_last, uint32_t per,
                uint32_t q0, const uint32_t *__restrict__ list, uint32_t nlist, uint32_t ublocks,
                int32_t *__restrict__ est) {
    extern __shared__ uint64_t tab[];
    const uint32_t tid = threadIdx.x;
    const uint32_t L = xcd_slice(blockIdx.x, gridDim.x);
    const uint64_t ubase = (uint64_t)(L % ublocks) * blockDim.x * kUPT;
    const uint32_t q_begin = q_first + (L / ublocks) * per;
    const uint32_t q_end = min(q_last, q_begin + per);
    // uniform: the whole workgroup leaves
    if (ubase >= nlist || q_begin >= q_end) return;
    uint32_t u[kUPT];
    int32_t cnt[kUPT];
#pragma unroll
    for (int k = 0; k < kUPT; ++k) {
        const uint64_t i = ubase + tid + (uint64_t)k * blockDim.x;
        u[k] = i < nlist ? list[i] : 0xffffffffu;
        cnt[k] = 0;
    }
    for (uint32_t qb = q_begin; qb < q_end; qb += kQB) {
        const uint32_t nqb = min((uint32_t)kQB, q_end - qb);
        uint64_t acc[kQB][kUPT];
#pragma unroll
        for (int a = 0; a < kQB; ++a) {
            // nodes past n in the last chunk never count
            const uint64_t first = (uint64_t)(qb + a) * 64;
            const uint64_t valid = (a < (int)nqb && first < n)
                                       ? ((n - first >= 64) ? ~0ull : ((1ull << (n - first)) - 1ull))
                                       : 0ull;
#pragma unroll
            for (int k = 0; k < kUPT; ++k) acc[a][k] = valid;
        }
        for (uint32_t j0 = 0; j0 < H; j0 += G) {
            const uint32_t g = min(G, H - j0);
            uint32_t b[kUPT][4];
            // buckets of this hash group (G <= 4)
#pragma unroll
            for (int k = 0; k < kUPT; ++k)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    b[k][jj] = (u[k] != 0xffffffffu && jj < (int)g) ? bucket[(size_t)(j0 + jj) * n + u[k]] : 0u;
#pragma unroll
            for (int a = 0; a < kQB; ++a) {
                if (a >= (int)nqb) break;
                const uint64_t *src = Lt + ((size_t)(qb + a - q0) * H + j0) * K;
                const uint64_t *tb = src;
                if (LDS) {
                    __syncthreads();
                    stage_tables(src, g * K, K, tab);
                    __syncthreads();
                    tb = tab;
                }
#pragma unroll
                for (int k = 0; k < kUPT; ++k)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        if (jj < (int)g) acc[a][k] &= tb[(size_t)jj * K + b[k][jj]];
            }
        }
#pragma unroll
        for (int a = 0; a < kQB; ++a)
#pragma unroll
            for (int k = 0; k < kUPT; ++k) cnt[k] += __popcll(acc[a][k]);
    }
#pragma unroll
    for (int k = 0; k < kUPT; ++k)
        if (u[k] != 0xffffffffu && cnt[k]) atomicAdd(est + u[k], cnt[k]);
}

// The same sums as k_recombine_est with LDS, for tables of GB hashes whose
// two copies fit in LDS together: while a stage (one chunk, one group of GB
// hashes) is read from one buffer, the next stage's tables stream into the
// other, and the next group's buckets are requested before them (loads
// retire in order, so they must not queue behind the tables).
template <int GB>
__global__ void __launch_bounds__(kRecombineThreads)
k_recombine_est2(uint32_t n, uint32_t H, uint32_t K, const uint32_t *__restrict__ bucket,
                 const uint64_t *__restrict__ Lt, uint32_t q_first, uint32_t q_last, uint32_t per,
                 uint32_t q0, const uint32_t *__restrict__ list, uint32_t nlist, uint32_t ublocks,
                 int32_t *__restrict__ est) {
    extern __shared__ uint64_t tab[];  // two buffers of GB K words
    const uint32_t tid = threadIdx.x;
    const uint32_t L = xcd_slice(blockIdx.x, gridDim.x);
    const uint64_t ubase = (uint64_t)(L % ublocks) * blockDim.x * kUPT;
    const uint32_t q_begin = q_first + (L / ublocks) * per;
    const uint32_t q_end = min(q_last, q_begin + per);
    // uniform: the whole workgroup leaves
    if (ubase >= nlist || q_begin >= q_end) return;
    uint32_t u[kUPT];
    int32_t cnt[kUPT];
#pragma unroll
    for (int k = 0; k < kUPT; ++k) {
        const uint64_t i = ubase + tid + (uint64_t)k * blockDim.x;
        u[k] = i < nlist ? list[i] : 0xffffffffu;
        cnt[k] = 0;
    }
    const uint32_t groups = (H + GB - 1) / GB;
    const size_t bufw = (size_t)GB * K;
    uint32_t bc[kUPT][GB], bn[kUPT][GB];
    auto load_buckets = [&](uint32_t (&b)[kUPT][GB], uint32_t grp) {
        const uint32_t g = min((uint32_t)GB, H - grp * GB);
#pragma unroll
        for (int k = 0; k < kUPT; ++k)
#pragma unroll
            for (int jj = 0; jj < GB; ++jj)
                b[k][jj] = (u[k] != 0xffffffffu && jj < (int)g)
                               ? bucket[(size_t)(grp * GB + jj) * n + u[k]]
                               : 0u;
    };
    load_buckets(bc, 0);
    stage_tables(Lt + (size_t)(q_begin - q0) * H * K, min((uint32_t)GB, H) * K, K, tab);
    uint32_t buf = 0;
    for (uint32_t qb = q_begin; qb < q_end; qb += kQB) {
        const uint32_t nqb = min((uint32_t)kQB, q_end - qb);
        uint64_t acc[kQB][kUPT];
#pragma unroll
        for (int a = 0; a < kQB; ++a) {
            // nodes past n in the last chunk never count
            const uint64_t first = (uint64_t)(qb + a) * 64;
            const uint64_t valid = (a < (int)nqb && first < n)
                                       ? ((n - first >= 64) ? ~0ull : ((1ull << (n - first)) - 1ull))
                                       : 0ull;
#pragma unroll
            for (int k = 0; k < kUPT; ++k) acc[a][k] = valid;
        }
        for (uint32_t grp = 0; grp < groups; ++grp) {
            const uint32_t g = min((uint32_t)GB, H - grp * GB);
#pragma unroll
            for (int a = 0; a < kQB; ++a) {
                if (a >= (int)nqb) break;
                // the stage after this one
                const bool last_a = a + 1 == (int)nqb;
                uint32_t qb2 = qb, grp2 = grp, a2 = a + 1;
                if (last_a) {
                    a2 = 0;
                    grp2 = grp + 1;
                    if (grp2 == groups) {
                        grp2 = 0;
                        qb2 = qb + kQB;
                    }
                }
                const bool more = qb2 < q_end;
                // this stage's tables are in, and every wave is done with
                // the other buffer
                __syncthreads();
                if (more && last_a) load_buckets(bn, grp2);
                if (more)
                    stage_tables(Lt + ((size_t)(qb2 + a2 - q0) * H + grp2 * GB) * K,
                                 min((uint32_t)GB, H - grp2 * GB) * K, K,
                                 tab + (buf ^ 1u) * bufw);
                const uint64_t *tb = tab + buf * bufw;
                if (g == GB) {
                    // a whole group: every read unconditional, so they can be
                    // in flight together
#pragma unroll
                    for (int k = 0; k < kUPT; ++k)
#pragma unroll
                        for (int jj = 0; jj < GB; ++jj)
                            acc[a][k] &= tb[(size_t)jj * K + bc[k][jj]];
                } else {
#pragma unroll
                    for (int k = 0; k < kUPT; ++k)
#pragma unroll
                        for (int jj = 0; jj < GB; ++jj)
                            if (jj < (int)g) acc[a][k] &= tb[(size_t)jj * K + bc[k][jj]];
                }
                if (more && last_a) {
                    // after this stage's reads: the next group's buckets
#pragma unroll
                    for (int k = 0; k < kUPT; ++k)
#pragma unroll
                        for (int jj = 0; jj < GB; ++jj)
                            asm volatile("" : "=v"(bc[k][jj]) : "0"(bn[k][jj]) : "memory");
                }
                buf ^= 1u;
            }
        }
#pragma unroll
        for (int a = 0; a < kQB; ++a)
#pragma unroll
            for (int k = 0; k < kUPT; ++k) cnt[k] += __popcll(acc[a][k]);
    }
#pragma unroll
    for (int k = 0; k < kUPT; ++k)
        if (u[k] != 0xffffffffu && cnt[k]) atomicAdd(est + u[k], cnt[k]);
}

uint32_t grid_for(size_t items, uint32_t per_block, uint32_t cap = 65536) {
    size_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

}  // namespace

hipError_t launch_hash_buckets(uint32_t n, uint32_t H, const uint64_t *coeffs, int order, uint32_t K,
                               uint32_t *bucket, int32_t *count, hipStream_t st) {
    const size_t total = (size_t)n * H;
    hipLaunchKernelGGL(k_hash_buckets, dim3(grid_for(total, 256)), dim3(256), 0, st, n, H, coeffs,
                       order, K, bucket);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for((size_t)H * K, 256)), dim3(256), 0, st, count,
                       (size_t)H * K);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bucket_counts, dim3(grid_for(total, 256)), dim3(256), 0, st, n, H, K,
                       bucket, count);
    return hipGetLastError();
}

hipError_t launch_transpose_proxies(uint32_t H, uint32_t K, int64_t ldK, const uint64_t *P,
                                    uint64_t *PT, hipStream_t st) {
    const size_t kw = (K + 63) / 64;
    const size_t runs = (kw + kLiftRun - 1) / kLiftRun;
    hipLaunchKernelGGL(k_transpose_proxies, dim3(grid_for((size_t)H * kw * runs * 64, 256)), dim3(256),
                       0, st, H, K, ldK, P, PT);
    return hipGetLastError();
}

hipError_t launch_row_sums_full(uint32_t H, uint32_t K, int64_t ldK, const uint64_t *P,
                               const int32_t *count, int32_t *bsum, int32_t *rowsum, uint8_t *full,
                               hipStream_t st) {
    const size_t kw = (K + 63) / 64;
    if (rowsum) {
        hipLaunchKernelGGL(k_block_sums, dim3(grid_for((size_t)H * kw * 64, 256)), dim3(256), 0, st,
                           H, K, count, bsum);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_row_sums_full, dim3(grid_for((size_t)H * K * 64, 256)), dim3(256), 0, st, H,
                       K, ldK, P, count, bsum, rowsum, full);
    return hipGetLastError();
}

hipError_t launch_lifted_sizes(uint32_t n, uint32_t H, uint32_t K, const uint32_t *bucket,
                               const int32_t *rowsum, int32_t *lifted, hipStream_t st) {
    hipLaunchKernelGGL(k_lifted_sizes, dim3(grid_for((size_t)n * H, 256)), dim3(256), 0, st, n, H,
                       bucket, rowsum, K, lifted);
    return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t *p, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_build_lifted(uint32_t n, uint32_t H, uint32_t K, int64_t ldK, const uint64_t *PT,
                               const uint32_t *bucket, uint32_t q0, uint32_t nq, uint64_t *Lt,
                               hipStream_t st) {
    const size_t kw = (K + 63) / 64;
    const size_t runs = (kw + kLiftRun - 1) / kLiftRun;
    hipLaunchKernelGGL(k_build_lifted, dim3(grid_for((size_t)nq * H * runs * 64, 256)), dim3(256), 0,
                       st, n, H, K, ldK, PT, bucket, q0, nq, Lt);
    return hipGetLastError();
}

// Hashes whose chunk tables fit in LDS together (at most 4); 0 when one
// table does not fit, and the tables are read from global memory.
uint32_t recombine_group(uint32_t K) {
    const size_t budget = kRecombineLds;
    size_t g = budget / ((size_t)K * 8);
    if (g > 4) g = 4;
    return (uint32_t)g;
}

hipError_t launch_split_full(uint32_t n, uint32_t H, uint32_t K, const uint32_t *bucket,
                             const uint8_t *full, int32_t *est, uint32_t *list, uint32_t *count,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, (int32_t *)count, (size_t)1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_split_full, dim3(grid_for(n, 256)), dim3(256), 0, st, n, H, K, bucket, full,
                       est, list, count);
    return hipGetLastError();
}

hipError_t launch_recombine_est(uint32_t n, uint32_t H, uint32_t K, const uint32_t *bucket,
                                const uint64_t *Lt, uint32_t q0, uint32_t nq, const uint32_t *list,
                                uint32_t nlist, int32_t *est, hipStream_t st) {
    const uint32_t GL = recombine_group(K);
    const bool in_lds = GL > 0;
    const uint32_t G = in_lds ? GL : 4u;
    // two copies of the tables of GB hashes when they fit (the next stage
    // streams in while this one is read), else one copy of G hashes, else
    // the tables are read where they are
    const uint32_t GB = (size_t)K * 8 * 2 * 2 <= kRecombineLds ? 2u
                      : (size_t)K * 8 * 2 <= kRecombineLds  ? 1u
                                                            : 0u;
    const size_t lds = GB ? (size_t)2 * GB * K * 8 : in_lds ? (size_t)G * K * 8 : 0;
    const void *kern = GB == 2 ? (const void *)k_recombine_est2<2>
                     : GB == 1 ? (const void *)k_recombine_est2<1>
                     : in_lds  ? (const void *)k_recombine_est<true>
                               : (const void *)k_recombine_est<false>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const uint32_t threads = kRecombineThreads;
    const uint32_t utiles = (uint32_t)((nlist + (size_t)threads * kUPT - 1) / ((size_t)threads * kUPT));
    if (utiles == 0) return hipSuccess;
    // split the chunk range over the second grid dimension so that the
    // launch has enough workgroups
    uint32_t splits = 1;
    while ((size_t)utiles * splits < 1024 && splits * kQB * 2 <= nq) splits *= 2;
    const uint32_t per = ((nq + splits - 1) / splits + kQB - 1) / kQB * kQB;
    splits = (nq + per - 1) / per;
    if (GB == 2)
        hipLaunchKernelGGL(k_recombine_est2<2>, dim3(utiles * splits), dim3(threads), lds, st, n, H,
                           K, bucket, Lt, q0, q0 + nq, per, q0, list, nlist, utiles, est);
    else if (GB == 1)
        hipLaunchKernelGGL(k_recombine_est2<1>, dim3(utiles * splits), dim3(threads), lds, st, n, H,
                           K, bucket, Lt, q0, q0 + nq, per, q0, list, nlist, utiles, est);
    else if (in_lds)
        hipLaunchKernelGGL(k_recombine_est<true>, dim3(utiles * splits), dim3(threads), lds, st, n,
                           H, K, G, bucket, Lt, q0, q0 + nq, per, q0, list, nlist, utiles, est);
    else
        hipLaunchKernelGGL(k_recombine_est<false>, dim3(utiles * splits), dim3(threads), lds, st, n,
                           H, K, G, bucket, Lt, q0, q0 + nq, per, q0, list, nlist, utiles, est);
    return hipGetLastError();
}

}  // namespace tn
