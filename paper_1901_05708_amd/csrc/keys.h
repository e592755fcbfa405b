// keys.h -- packed (value, index) keys used for the row / column minima.
//
// A global key is a 64-bit unsigned integer whose high bits are the bit
// pattern of a non-negative double x (the quantity being minimised) and whose
// low gb bits are replaced by a window index. For x >= +0 the unsigned order of
// the bit patterns is the order of the values, so one 64-bit atomicMin keeps
// both the minimum and its argument. Dropping gb mantissa bits bounds the
// relative precision of the comparison by 2^-(52-gb); the value reported for
// the winner is always recomputed exactly afterwards.
//
//   AAMP / p-norm : x = the pre-root sum S (Sec. 3.2: compare squares,
//                   take the root once at the end)
//   ACAMP         : x = 1 - rho, so DZ^2 = 2m x (Lemma 3, Eq. 8)
//
// ~0 (all ones) means "no candidate".
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpk {

constexpr unsigned long long KEY_NONE = ~0ull;

__device__ __forceinline__ unsigned long long pack_key(double x, unsigned long long idx,
                                                       unsigned long long mask)
{
    // clamp to +0 (negative round-off near a perfect match, and -0); a NaN,
    // which finite inputs never produce, ranks like +inf
    unsigned long long b = (x > 0.0)    ? (unsigned long long)__double_as_longlong(x)
                           : (x <= 0.0) ? 0ull
                                        : 0x7FF0000000000000ull;
    return (b & ~mask) | idx;
}

__device__ __forceinline__ double key_value(unsigned long long key, unsigned long long mask)
{
    return __longlong_as_double((long long)(key & ~mask));
}

}  // namespace mpk
