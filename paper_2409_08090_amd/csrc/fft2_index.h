// fft2_index.h -- index arithmetic of the two-pass register-tile FFT
// (host and device; no HIP dependency, so a host build can check it).
//
// A grid of n = L0 * L1 cells, cell l = l0 * L1 + s (row l0 < L0, column
// s < L1), is transformed (sign +, unnormalised) in two passes:
//   first pass: length-L0 transforms down each column s, output digit m0,
//     multiplied by exp(2 pi i s m0 / n), stored row-major: element
//     (s, m0) at m0 * L1 + s (a workgroup of C columns writes C-element
//     pieces of every row);
//   last pass: length-L1 transforms along each row m0 of that result,
//     output digit m1; mode m = m0 + L0 m1.
// Each transform of length L = 16^k f (f in {1, 2, 4, 8}) is held in the
// registers of L / 16 threads, 16 elements per thread, and runs as Stockham
// stages of radix 16 (then one of radix f): in stage s of radix R, after
// stages whose radices multiply to Ns, butterfly b takes the elements at
// positions b + q (L / R), q < R, multiplies element q by
// exp(2 pi i q (b mod Ns) / (Ns R)), takes the length-R DFT and leaves
// output q at (b / Ns) Ns R + (b mod Ns) + q Ns.  Thread t of a line holds
// the butterflies b = t + (L/16) k, k < 16 / R, in registers v[k R + q];
// between stages the elements move through LDS.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define F2_HD __host__ __device__
#else
#define F2_HD
#endif

namespace mils {
namespace fft2 {

// lengths supported by a register-tile line: 16^k f, k >= 2, f in {1,2,4,8}
F2_HD constexpr bool line_ok(int L) {
  return L == 256 || L == 512 || L == 1024 || L == 2048 || L == 4096 || L == 8192;
}
// number of stages and the radix of stage s (radix 16 first)
F2_HD constexpr int n16(int L) { return L >= 4096 ? 3 : 2; }
F2_HD constexpr int tailr(int L) {
  return L == 512 || L == 8192 ? 2 : (L == 1024 ? 4 : (L == 2048 ? 8 : 1));
}
F2_HD constexpr int nstages(int L) { return n16(L) + (tailr(L) > 1 ? 1 : 0); }
F2_HD constexpr int radix(int L, int s) { return s < n16(L) ? 16 : tailr(L); }
// product of the radices of the stages before s
F2_HD constexpr int ns(int L, int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= radix(L, i);
  return p;
}
// threads of one line
F2_HD constexpr int threads(int L) { return L / 16; }

// position of input q of butterfly b in stage s
F2_HD constexpr int in_pos(int L, int s, int b, int q) { return b + q * (L / radix(L, s)); }
// position of output q of butterfly b in stage s
F2_HD constexpr int out_pos(int L, int s, int b, int q) {
  return (b / ns(L, s)) * ns(L, s) * radix(L, s) + (b % ns(L, s)) + q * ns(L, s);
}
// register of element q of the thread's butterfly k in stage s
F2_HD constexpr int reg(int L, int s, int k, int q) { return k * radix(L, s) + q; }
// after the last stage register r holds output index t + (L/16) j(r)
F2_HD constexpr int final_j(int L, int r) {
  return (r % radix(L, nstages(L) - 1)) * (16 / radix(L, nstages(L) - 1)) +
         r / radix(L, nstages(L) - 1);
}
// LDS slot of position p of a line: one pad element per 16
F2_HD constexpr int pad(int p) { return p + (p >> 4); }
// LDS elements per line (pads, plus 8 so that consecutive lines start on
// different banks)
F2_HD constexpr int line_pitch(int L) { return L + L / 16 + 8; }
// pitch of the C lines of a first-pass workgroup, whose lanes take the C
// columns fastest: with lines 16 / C elements apart modulo 16, the 16 lanes
// of one LDS access cycle (C columns x 16 / C threads, 8-byte elements) fall
// on distinct bank pairs
F2_HD constexpr int line_pitch_c(int L, int C) { return L + L / 16 + (C >= 2 ? 16 / C : 8); }

// output index (0 .. nf-1) of mode m of an n-cell grid, or -1 when cropped:
// modes m <= nf-1-K are the non-negative ones, m >= n-K the negative ones
F2_HD inline int64_t crop(int64_t m, int64_t n, int64_t nf, int64_t K) {
  const int64_t mm = m <= nf - 1 - K ? m : m - n;
  const int64_t k = mm + K;
  return (k >= 0 && k < nf) ? k : -1;
}

}  // namespace fft2
}  // namespace mils
