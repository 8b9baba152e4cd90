// Device helpers shared by the kernels that merge HyperLogLog registers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tn {

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
