// Exact uint64 arithmetic of the DP with the overflow rule: every result is
// the residue mod 2^64, and a flag records whether the exact value reached
// 2^64.  Written for the device; plain C++ otherwise, so a host compiler can
// check it against 128-bit arithmetic (include it after the HIP runtime
// header on the device side).
#pragma once

#include <cstdint>

namespace sc {
namespace kern {

// acc + a*b mod 2^64; sets `ovf` when a*b >= 2^64 (the high half of the
// 128-bit product is non-zero) or the sum carries.  A split into 32-bit
// halves needing only three multiplies was measured slower in the row
// kernels: it raises register use more than it saves.
__host__ __device__ __forceinline__ uint64_t mad_ovf(uint64_t acc, uint64_t a, uint64_t b,
                                                     uint32_t &ovf) {
    const unsigned __int128 p = (unsigned __int128)a * b;
    const uint64_t lo = (uint64_t)p;
    const uint64_t s = acc + lo;
    ovf |= (uint32_t)((uint64_t)(p >> 64) != 0) | (uint32_t)(s < lo);
    return s;
}

}  // namespace kern
}  // namespace sc
