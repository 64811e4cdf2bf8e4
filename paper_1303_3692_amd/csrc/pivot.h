// Pivot rule of the binary searches (Section IV, Algorithm 1), shared by
// the device kernels and the host code that builds the LDS tile.  Plain
// C++ so that a CPU test can check it at the largest text length.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define SAMATCH_HD __host__ __device__
#else
#define SAMATCH_HD
#endif

namespace samatch {

// Row halfway through the open range (L, R), -1 <= L < R <= 2^31 - 1.  The
// paper's (L + R) / 2 overflows 32 bits near n = 2^31, and so does R - L
// in signed arithmetic (L = -1, R = 2^31 - 1); the difference is taken in
// unsigned arithmetic, where it always fits, and half of it keeps L + d
// within [L, R].
SAMATCH_HD inline int midpoint(int L, int R) {
    return L + (int)(((uint32_t)R - (uint32_t)L) >> 1);
}

}  // namespace samatch
