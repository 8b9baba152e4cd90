// Launchers of the hashing and fusion kernels (tn_hash.hip).
#pragma once

#include "tn_internal.h"

namespace tn {

hipError_t launch_hash_buckets(uint32_t n, uint32_t H, const uint64_t *coeffs, int order, uint32_t K,
                               uint32_t *bucket, int32_t *count, hipStream_t st);
hipError_t launch_transpose_proxies(uint32_t H, uint32_t K, int64_t ldK, const uint64_t *P,
                                    uint64_t *PT, hipStream_t st);
// full[j K + r] = 1 iff proxy row r of P_j is full; with rowsum, also the
// lifted row sums rowsum[j K + r] (bsum: scratch of H ceil(K/64) int32).
hipError_t launch_row_sums_full(uint32_t H, uint32_t K, int64_t ldK, const uint64_t *P,
                               const int32_t *count, int32_t *bsum, int32_t *rowsum, uint8_t *full,
                               hipStream_t st);
// lifted[j n + u] = rowsum[j K + h_j(u)].
hipError_t launch_lifted_sizes(uint32_t n, uint32_t H, uint32_t K, const uint32_t *bucket,
                               const int32_t *rowsum, int32_t *lifted, hipStream_t st);
hipError_t launch_zero_i32(int32_t *p, size_t n, hipStream_t st);
hipError_t launch_build_lifted(uint32_t n, uint32_t H, uint32_t K, int64_t ldK, const uint64_t *PT,
                               const uint32_t *bucket, uint32_t q0, uint32_t nq, uint64_t *Lt,
                               hipStream_t st);
// est[u] = n for nodes whose proxy rows are full in every hash (full from
// launch_row_sums_full); the others get est[u] = 0 and are listed in
// list[0 .. *count).
hipError_t launch_split_full(uint32_t n, uint32_t H, uint32_t K, const uint32_t *bucket,
                             const uint8_t *full, int32_t *est, uint32_t *list, uint32_t *count,
                             hipStream_t st);
hipError_t launch_recombine_est(uint32_t n, uint32_t H, uint32_t K, const uint32_t *bucket,
                                const uint64_t *Lt, uint32_t q0, uint32_t nq, const uint32_t *list,
                                uint32_t nlist, int32_t *est, hipStream_t st);
uint32_t recombine_group(uint32_t K);

}  // namespace tn
