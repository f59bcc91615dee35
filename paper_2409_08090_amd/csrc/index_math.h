// index_math.h -- 32-bit index arithmetic of the binning, written once for the
// kernels and for a host build that checks it at the largest accepted point
// count (kMaxPoints).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define MILS_HD __host__ __device__
#else
#define MILS_HD
#endif

namespace mils {

// Largest accepted number of points.  Every point index, every bin start
// and every loop bound of the binning and spreading kernels is a 32-bit int;
// with n <= 2^30, index + blockDim (<= 1024) and lo + (hi - lo) / 2 stay
// below 2^31.
constexpr int64_t kMaxPoints = (int64_t)1 << 30;

// First index j in [0, n) with key_at(j) >= b, or n if there is none
// (key_at non-decreasing).  The midpoint is formed without lo + hi.
template <typename KeyAt>
MILS_HD inline int lower_bound_idx(int n, int b, KeyAt key_at) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = lo + ((hi - lo) >> 1);
    if (key_at(mid) < b) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

}  // namespace mils
