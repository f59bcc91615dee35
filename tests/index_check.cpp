// Host build of the binning's 32-bit index arithmetic (index_math.h) at the
// largest point counts: prints one line per case, "ok" or the mismatch.
#include <cstdint>
#include <cstdio>

#include "../paper_2409_08090_amd/csrc/index_math.h"

using mils::lower_bound_idx;

// keys of a virtual sorted array: key(j) = j / 32 (bins of 32 points),
// nothing stored
static int check(int n, int b) {
  const int got = lower_bound_idx(n, b, [](int j) { return j >> 5; });
  const int64_t want64 = (int64_t)b * 32;
  const int want = want64 > n ? n : (int)want64;
  if (got != want) {
    std::printf("n=%d b=%d got=%d want=%d\n", n, b, got, want);
    return 1;
  }
  return 0;
}

int main() {
  int bad = 0;
  const int nmax = (int)mils::kMaxPoints;  // 2^30
  const int cases_n[] = {1, 2, 33, nmax - 1, nmax, 2147483647};
  for (int n : cases_n) {
    const int last_bin = (int)(((int64_t)n - 1) >> 5);
    const int bs[] = {0, 1, last_bin - 1, last_bin, last_bin + 1, last_bin + 1000};
    for (int b : bs)
      if (b >= 0) bad += check(n, b);
  }
  // the spread's chunk loop: base = start; base < end; base += 1024 never
  // wraps for end <= kMaxPoints
  int64_t last = 0;
  for (int64_t base = nmax - 5000; base < nmax; base += 1024) last = base + 1024;
  if (last > 2147483647LL) {
    std::printf("chunk loop bound overflows\n");
    ++bad;
  }
  std::printf(bad ? "FAIL %d\n" : "ok\n", bad);
  return bad ? 1 : 0;
}
