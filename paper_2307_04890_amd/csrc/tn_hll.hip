// HyperLogLog structures of the reverse-time stream (Sec. 3.4, with the HLL
// of Sec. 2.2): every node holds s = 2^b one-byte registers, the structure
// of the set {node} at first; the stream merges structures with the
// register-wise maximum (launch_rowmax_global, the row-OR kernel's level
// loop on rows of s bytes, or launch_hll_levels below, one launch per level
// of a TN_HLL plan); the estimate of each row follows Flajolet,
// Fusy, Gandouet and Meunier (2007): alpha_s s^2 / sum_j 2^-M[j], and
// s ln(s / V) when that is at most 5s/2 with V > 0 zero registers.
// Element hashes are inputs, one uniform 64-bit value per node.
#include <hip/hip_runtime.h>

#include "tn_device.h"
#include "tn_internal.h"

namespace tn {

namespace {

// Row u = the registers of {u}: register j (the top b bits of the hash)
// holds rho, the 1-based position of the leftmost 1 in the other 64 - b
// bits (64 - b + 1 when they are all zero).  One thread per word.
__global__ void __launch_bounds__(256)
k_hll_init(uint32_t n, uint32_t b, const uint64_t *__restrict__ node_hash, uint64_t *__restrict__ M) {
    const uint32_t nwords = (1u << b) / 8;
    const size_t total = (size_t)n * nwords;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t u = (uint32_t)(i / nwords), w = (uint32_t)(i % nwords);
        const uint64_t x = node_hash[u];
        const uint32_t j = (uint32_t)(x >> (64 - b));
        const uint64_t tail = x & ((~0ull) >> b);
        const uint32_t rho = tail ? (uint32_t)__clzll((long long)tail) - b + 1 : 64 - b + 1;
        M[i] = (j >> 3) == w ? (uint64_t)rho << (8 * (j & 7u)) : 0ull;
    }
}

// Lane values of LW words and their register-wise maximum.
template <int LW>
__device__ __forceinline__ typename LaneT<LW>::T max_lane(typename LaneT<LW>::T a,
                                                          typename LaneT<LW>::T b) {
    if constexpr (LW == 1) {
        return max_bytes7(a, b);
    } else {
        typename LaneT<LW>::T r;
        r.x = max_bytes7(a.x, b.x);
        r.y = max_bytes7(a.y, b.y);
        return r;
    }
}

// One level of the register stream of a TN_HLL plan.  Items [0, np) are
// the level's pairs: both rows (one for a one-way pair) become their
// register-wise maximum, in place (the items of a level touch disjoint
// rows).  The level's gathers read each other's rows (those of one compound
// item), so every source is read before any target is written:
//  - a level with at most hll_block_gathers(G) gathers (nearly all of them)
//    hands them to one extra workgroup, the grid's last: each of its lane
//    groups reads the sources of its gathers into scratch rows, a barrier
//    of the workgroup ends every read, then each group writes its targets;
//  - else items [np, np + ng) are the gathers, each writing scratch row
//    i - np, and k_hll_gathers_write copies them in a launch of its own.
// A group of G lanes takes an item; lane k takes LW words at LW k,
// LW (k + G), ... of its rows, so each row access is one contiguous segment
// (LW = 2: 16-byte accesses, half the wave instructions of LW = 1).
//
// A gather's sources are read four at a time (indices, then rows, each
// four independent loads); a short last batch repeats its last source,
// which the maximum ignores.
template <int LW>
__device__ __forceinline__ void hll_gather_read(const uint64_t *__restrict__ M, uint32_t nwords,
                                                uint32_t lane, uint32_t G, uint32_t s0, uint32_t s1,
                                                const uint32_t *__restrict__ gat_src,
                                                uint64_t *__restrict__ dst) {
    using T = typename LaneT<LW>::T;
    for (uint32_t w = lane * LW; w < nwords; w += G * LW) {
        T acc = {};  // registers are never negative
        for (uint32_t q = s0; q < s1; q += 4) {
            uint32_t id[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) id[k] = gat_src[min(q + k, s1 - 1)];
            T r[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) r[k] = *(const T *)(M + (size_t)id[k] * nwords + w);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc = max_lane<LW>(acc, r[k]);
        }
        *(T *)(dst + w) = acc;
    }
}

// Saturation.  No row can exceed G, the register-wise maximum over every
// node's own registers (every row is the maximum over a set of nodes), and
// a row equal to G stays G.  *left counts the rows not yet equal to G: each
// row that reaches G takes one off (a row does so once), and once it is 0
// the rest of the stream changes nothing, so every later level returns at
// once.  `all` over a group of G lanes: each lane folds its own words, then
// a ballot over the group's lanes.
__device__ __forceinline__ bool group_all(bool mine, uint32_t G) {
    const uint64_t b = __ballot(mine);
    const uint32_t first = (threadIdx.x & 63u) / G * G;
    const uint64_t mask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << first;
    return (b & mask) == mask;
}

// Target g of a level's gathers takes scratch row g; with saturation, a
// target that reaches G takes one off *left (whole groups run this, so the
// ballots see every lane of the group).
template <int LW>
__device__ __forceinline__ void hll_gather_write(uint64_t *__restrict__ M, uint32_t nwords,
                                                 uint32_t lane, uint32_t G, uint32_t tgt,
                                                 const uint64_t *__restrict__ srow,
                                                 const uint64_t *__restrict__ Grow,
                                                 unsigned int *__restrict__ left) {
    using T = typename LaneT<LW>::T;
    bool was = true, is = true;
    for (uint32_t w = lane * LW; w < nwords; w += G * LW) {
        T *tp = (T *)(M + (size_t)tgt * nwords + w);
        const T old = *tp;
        const T nw = *(const T *)(srow + w);
        T gw = {};
        if (Grow) gw = *(const T *)(Grow + w);
        *tp = nw;
        if (Grow) {
            was &= lane_eq<LW>(old, gw);
            is &= lane_eq<LW>(nw, gw);
        }
    }
    if (Grow) {
        const bool reached = group_all(is, G), before = group_all(was, G);
        if (reached && !before && lane == 0) atomicSub(left, 1u);
    }
}

// Gathers one workgroup of 256 threads takes: four per lane group.
__host__ __device__ constexpr uint32_t hll_block_gathers(uint32_t G) { return 4u * (256u / G); }

template <int LW>
__global__ void __launch_bounds__(256)
k_hll_level(uint64_t *__restrict__ M, uint32_t nwords, uint32_t G, const uint2 *__restrict__ pairs,
            uint32_t np, const uint32_t *__restrict__ gat_ptr,
            const uint32_t *__restrict__ gat_src, const uint32_t *__restrict__ gat_tgt,
            uint32_t ng, uint32_t block_gathers, uint64_t *__restrict__ scr,
            const uint64_t *__restrict__ Grow, unsigned int *__restrict__ left) {
    using T = typename LaneT<LW>::T;
    const uint32_t lane = threadIdx.x % G;
    const uint32_t grp = threadIdx.x / G, ngr = blockDim.x / G;
    const bool gblock = block_gathers && ng > 0;
    const uint32_t pblocks = gridDim.x - (gblock ? 1u : 0u);
    if (blockIdx.x == pblocks) {
        // the level's gathers (the launcher adds this block only when they
        // number at most hll_block_gathers(G))
        uint32_t tg[4], s0[4], s1[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t g = min(grp + k * ngr, ng - 1);
            tg[k] = gat_tgt[g];
            s0[k] = gat_ptr[g];
            s1[k] = gat_ptr[g + 1];
        }
        if (left && __builtin_amdgcn_readfirstlane(*left) == 0u) return;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t g = grp + k * ngr;
            if (g < ng)
                hll_gather_read<LW>(M, nwords, lane, G, s0[k], s1[k], gat_src,
                                    scr + (size_t)g * nwords);
        }
        // every source of the level is read before any target is written
        // (a lane reads back only the scratch words it wrote itself)
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t g = grp + k * ngr;
            if (g < ng)
                hll_gather_write<LW>(M, nwords, lane, G, tg[k], scr + (size_t)g * nwords, Grow,
                                     left);
        }
        return;
    }
    const uint32_t ngroups = pblocks * ngr;
    const uint32_t items = np + (gblock ? 0u : ng);
    const uint32_t i0 = blockIdx.x * ngr + grp;
    // the first pair is requested before the count is tested, so that the
    // two reads overlap (the count's wait is on the scalar counter only)
    uint2 first = make_uint2(0u, 0u);
    if (i0 < np) first = pairs[i0];
    // every row is G: nothing changes (one read per wavefront, so that its
    // lanes leave together)
    if (left && __builtin_amdgcn_readfirstlane(*left) == 0u) return;
    // groups never straddle a wavefront (G divides 64), and every lane of a
    // group runs the same iterations, so the ballots below see whole groups
    const uint32_t rounds = (items + ngroups - 1) / ngroups;
    for (uint32_t rr = 0; rr < rounds; ++rr) {
        const uint32_t i = i0 + rr * ngroups;
        bool ru_was = true, rv_was = true, r_is = true, one_way = true, pair = false;
        if (i >= items) {
            // no item: takes part in the ballots only
        } else if (i < np) {
            const uint2 it = rr == 0 ? first : pairs[i];
            const uint32_t v = it.y & kNodeMask;
            const bool dir = it.y & kDirBit;
            uint64_t *ru = M + (size_t)it.x * nwords;
            uint64_t *rv = M + (size_t)v * nwords;
            pair = true;
            one_way = dir;
            for (uint32_t w = lane * LW; w < nwords; w += G * LW) {
                const T a = *(const T *)(ru + w), b = *(const T *)(rv + w);
                // G is read with the rows, not after the stores: loads and
                // stores retire in order, so a later read would wait for them
                T gw = {};
                if (Grow) gw = *(const T *)(Grow + w);
                const T r = max_lane<LW>(a, b);
                *(T *)(ru + w) = r;
                if (!dir) *(T *)(rv + w) = r;
                if (Grow) {
                    ru_was &= lane_eq<LW>(a, gw);
                    rv_was &= lane_eq<LW>(b, gw);
                    r_is &= lane_eq<LW>(r, gw);
                }
            }
        } else {
            const uint32_t g = i - np;
            hll_gather_read<LW>(M, nwords, lane, G, gat_ptr[g], gat_ptr[g + 1], gat_src,
                                scr + (size_t)g * nwords);
        }
        if (Grow) {
            const bool is = group_all(r_is, G);
            const bool u_was = group_all(ru_was, G), v_was = group_all(rv_was, G);
            if (pair && lane == 0 && is) {
                const unsigned int k = (u_was ? 0u : 1u) + ((one_way || v_was) ? 0u : 1u);
                if (k) atomicSub(left, k);
            }
        }
    }
}

// The level's gathers write their targets from scratch, one group of G
// lanes per target (so that a target reaching G is counted once).
template <int LW>
__global__ void __launch_bounds__(256)
k_hll_gathers_write(uint64_t *__restrict__ M, uint32_t nwords, uint32_t G,
                    const uint32_t *__restrict__ gat_tgt, uint32_t ng,
                    const uint64_t *__restrict__ scr, const uint64_t *__restrict__ Grow,
                    unsigned int *__restrict__ left) {
    // every row is G: the level changes nothing, and its gather launch may
    // have left scratch unwritten (the count only falls, so a count above 0
    // here means the gather launch before saw one too and wrote all of it)
    if (left && __builtin_amdgcn_readfirstlane(*left) == 0u) return;
    const uint32_t lane = threadIdx.x % G;
    const uint32_t ngroups = gridDim.x * (blockDim.x / G);
    const uint32_t g0 = blockIdx.x * (blockDim.x / G) + threadIdx.x / G;
    // groups whose index passes ng have nothing to do: whole groups leave
    for (uint32_t g = g0; g < ng; g += ngroups)
        hll_gather_write<LW>(M, nwords, lane, G, gat_tgt[g], scr + (size_t)g * nwords, Grow, left);
}

// gmax[j] = the largest register j over every node's own registers.
__global__ void __launch_bounds__(256)
k_hll_gmax(uint32_t n, uint32_t b, const uint64_t *__restrict__ node_hash,
           unsigned int *__restrict__ gmax) {
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        const uint64_t x = node_hash[u];
        const uint32_t j = (uint32_t)(x >> (64 - b));
        const uint64_t tail = x & ((~0ull) >> b);
        const uint32_t rho = tail ? (uint32_t)__clzll((long long)tail) - b + 1 : 64 - b + 1;
        atomicMax(gmax + j, rho);
    }
}

// The row G from gmax, one byte per register.
__global__ void __launch_bounds__(256)
k_hll_pack_g(uint32_t nwords, const unsigned int *__restrict__ gmax, uint64_t *__restrict__ Grow) {
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += gridDim.x * blockDim.x) {
        uint64_t x = 0;
        for (uint32_t k = 0; k < 8; ++k) x |= (uint64_t)(gmax[8 * w + k] & 0xffu) << (8 * k);
        Grow[w] = x;
    }
}

// *left = the rows not equal to G (one wavefront per row).
__global__ void __launch_bounds__(256)
k_hll_count_left(uint32_t n, uint32_t nwords, const uint64_t *__restrict__ M,
                 const uint64_t *__restrict__ Grow, unsigned int *__restrict__ left) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwave = (gridDim.x * blockDim.x) >> 6;
    unsigned int mine = 0;
    for (uint32_t u = wave; u < n; u += nwave) {
        bool eq = true;
        for (uint32_t w = lane; w < nwords; w += 64) eq &= M[(size_t)u * nwords + w] == Grow[w];
        if (__ballot(!eq) != 0 && lane == 0) ++mine;
    }
    if (lane == 0 && mine) atomicAdd(left, mine);
}

double __device__ hll_alpha(uint32_t s) {
    if (s == 16) return 0.673;
    if (s == 32) return 0.697;
    if (s == 64) return 0.709;
    return 0.7213 / (1.0 + 1.079 / (double)s);
}

// One wavefront per node: the lanes sum 2^-M[j] and count zero registers,
// then lane 0 forms the estimate (double precision).
__global__ void __launch_bounds__(256)
k_hll_estimate(uint32_t n, uint32_t b, const uint8_t *__restrict__ M, double *__restrict__ est) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t s = 1u << b;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwave = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t u = wave; u < n; u += nwave) {
        const uint8_t *row = M + (size_t)u * s;
        double z = 0.0;
        uint32_t zeros = 0;
        for (uint32_t j = lane; j < s; j += 64) {
            const uint32_t r = row[j];
            z += ldexp(1.0, -(int)r);
            zeros += r == 0;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            z += __shfl_xor(z, off, 64);
            zeros += __shfl_xor(zeros, off, 64);
        }
        if (lane == 0) {
            const double sd = (double)s;
            double e = hll_alpha(s) * sd * sd / z;
            if (e <= 2.5 * sd && zeros > 0) e = sd * log(sd / (double)zeros);
            est[u] = e;
        }
    }
}

}  // namespace

hipError_t launch_hll_init(uint32_t n, uint32_t log2s, const uint64_t *node_hash, uint8_t *M,
                           hipStream_t st) {
    const size_t total = (size_t)n * ((1u << log2s) / 8);
    uint32_t blocks = (uint32_t)std::min<size_t>((total + 255) / 256, 65536);
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_hll_init, dim3(blocks), dim3(256), 0, st, n, log2s, node_hash,
                       (uint64_t *)M);
    return hipGetLastError();
}

hipError_t launch_hll_saturation_setup(uint32_t n, uint32_t log2s, const uint64_t *node_hash,
                                       const uint8_t *M, unsigned int *gmax, uint64_t *Grow,
                                       unsigned int *left, hipStream_t st) {
    const uint32_t s = 1u << log2s, nwords = s / 8;
    hipError_t e = launch_fill_u32(gmax, s, 0u, st);
    if (e == hipSuccess) e = launch_fill_u32(left, 1, 0u, st);
    if (e != hipSuccess) return e;
    uint32_t blocks = (n + 255) / 256;
    if (blocks > 4096u) blocks = 4096u;
    hipLaunchKernelGGL(k_hll_gmax, dim3(blocks), dim3(256), 0, st, n, log2s, node_hash, gmax);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hll_pack_g, dim3((nwords + 255) / 256), dim3(256), 0, st, nwords, gmax, Grow);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t cb = (n + 3) / 4;
    if (cb > 16384u) cb = 16384u;
    hipLaunchKernelGGL(k_hll_count_left, dim3(cb), dim3(256), 0, st, n, nwords,
                       (const uint64_t *)M, Grow, left);
    return hipGetLastError();
}

hipError_t launch_hll_levels(const DevSchedule &s, const uint32_t *lvl_pair,
                             const uint32_t *lvl_gat, uint32_t l0, uint32_t l1, uint32_t nwords,
                             uint64_t *M, uint64_t *scratch, const uint64_t *Grow,
                             unsigned int *left, hipStream_t st) {
    // two words per lane (nwords is a power of two >= 2, rows, scratch rows
    // and G start on 16 bytes), a group of at most 64 lanes per item
    constexpr int LW = 2;
    const uint32_t G = nwords / LW < 64 ? nwords / LW : 64;
    for (uint32_t l = l0; l < l1 && l < s.L; ++l) {
        const uint32_t p0 = lvl_pair[l], np = lvl_pair[l + 1] - p0;
        const uint32_t g0 = lvl_gat[l], ng = lvl_gat[l + 1] - g0;
        if (np + ng == 0) continue;
        // up to hll_block_gathers(G) gathers run in one extra workgroup of
        // the level's launch; more are spread over groups, then written by a
        // second launch
        const uint32_t inl = ng <= hll_block_gathers(G) ? 1u : 0u;
        const size_t threads = (size_t)(np + (inl ? 0u : ng)) * G;
        const uint32_t blocks = (uint32_t)std::min<size_t>((threads + 255) / 256, 4096) +
                                (inl && ng > 0 ? 1u : 0u);
        hipLaunchKernelGGL(k_hll_level<LW>, dim3(blocks), dim3(256), 0, st, M, nwords, G,
                           s.pairs + p0, np, s.gat_ptr + g0, s.gat_src, s.gat_tgt + g0, ng, inl,
                           scratch, Grow, left);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (ng == 0 || inl) continue;
        const size_t gthreads = (size_t)ng * G;
        const uint32_t wb = (uint32_t)std::min<size_t>((gthreads + 255) / 256, 4096);
        hipLaunchKernelGGL(k_hll_gathers_write<LW>, dim3(wb), dim3(256), 0, st, M, nwords, G,
                           s.gat_tgt + g0, ng, scratch, Grow, left);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_hll_estimate(uint32_t n, uint32_t log2s, const uint8_t *M, double *est,
                               hipStream_t st) {
    uint32_t blocks = (n + 3) / 4;
    if (blocks > 16384u) blocks = 16384u;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_hll_estimate, dim3(blocks), dim3(256), 0, st, n, log2s, M, est);
    return hipGetLastError();
}

}  // namespace tn
