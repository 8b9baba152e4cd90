// Device helpers shared by the row-OR kernels and those that merge
// HyperLogLog registers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tn {

// One op {a, b, d1, d2} as a native 4-lane vector.
typedef uint32_t op4 __attribute__((ext_vector_type(4)));

// Workgroups are dispatched round-robin over the 8 XCDs of the chip; map the
// workgroup index so that each XCD receives a contiguous range of slices
// (adjacent slices share cache lines of the same rows).
__device__ __forceinline__ uint32_t xcd_slice(uint32_t b, uint32_t nb) {
    const uint32_t x = b & 7u, k = b >> 3;
    const uint32_t q = nb >> 3, r = nb & 7u;
    return x * q + min(x, r) + k;
}


// A lane's words of a row: one (8-byte accesses) or two (16-byte accesses:
// per wave instruction twice the bytes for the same address work, which is
// what the texture address and data units of a CU spend their cycles on
// when 64 lanes touch 8 to 16 scattered row segments).
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
template <int LW>
struct LaneT;
template <>
struct LaneT<1> {
    using T = uint64_t;
};
template <>
struct LaneT<2> {
    using T = u64x2;
};

// Whether two lane values are equal in every word.
template <int LW>
__device__ __forceinline__ bool lane_eq(typename LaneT<LW>::T a, typename LaneT<LW>::T b) {
    if constexpr (LW == 1) {
        return a == b;
    } else {
        return a.x == b.x && a.y == b.y;
    }
}

// Byte-wise maximum of two words whose bytes are all below 128 (HyperLogLog
// registers, Sec. 3.4): (x | 0x80..) - y keeps each byte's borrow inside the
// byte, and that byte's top bit then says whether x >= y.
__device__ __forceinline__ uint64_t max_bytes7(uint64_t x, uint64_t y) {
    constexpr uint64_t H = 0x8080808080808080ull;
    const uint64_t ge = ((x | H) - y) & H;
    const uint64_t mask = (ge >> 7) * 0xFFull;
    return (x & mask) | (y & ~mask);
}

}  // namespace tn
