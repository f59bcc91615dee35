// fft2.h -- the two-pass register-tile FFT (device side): the first pass
// transforms the columns of a workgroup's column block, the last pass one
// row of each grid together with deconvolution, crop and power, and a tiled
// transpose puts the results in frequency order.  Index arithmetic and the
// stage structure are in fft2_index.h.
//
// Why this shape on gfx950: a 1.6e7-cell grid needs lines of ~4096 elements
// in each of two passes, and 4 columns x 4096 complex doubles (256 KB) do
// not fit the 160 KB of LDS.  So each thread keeps 16 elements in registers
// and the LDS only carries the exchange between radix-16 stages, one half
// (real or imaginary parts) at a time when a whole tile would not fit.  The
// first pass writes its result row-major, a piece of C elements of each row
// per workgroup, so that the last pass reads whole rows contiguously (the
// other way round -- column blocks stored contiguously, the last pass reading
// 64-byte pieces -- made the last pass, which has one workgroup per CU and
// waits for its loads, 426 us instead of 328 at 4096 x 4096 in FP64); the
// last pass holds one row per workgroup, so its results are written row by
// row and transposed by a separate tiled kernel (scattered 8-byte stores of
// the power cost more than the transpose).
#pragma once

#include "fft2_index.h"
#include "fft_core.h"
#include "path_device.h"

namespace mils {

// exp(2 pi i x / L), two-level table in LDS: lo[x mod 64] * hi[x / 64]
template <typename T2>
__device__ __forceinline__ T2 tw2(const T2* t, int x) {
  return cmul(t[kTwLo + (x >> 6)], t[x & (kTwLo - 1)]);
}

// Stage S of a line of length L: twiddles and the radix-R DFTs of the
// thread's butterflies (registers v).
template <int L, int S, typename T2>
__device__ __forceinline__ void f2_stage(T2 (&v)[16], int t, const T2* twl) {
  constexpr int R = fft2::radix(L, S), NS = fft2::ns(L, S), NB = 16 / R, TL = fft2::threads(L);
  constexpr int step = L / (NS * R);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if constexpr (NS > 1) {
      // exp(2 pi i q kb / (NS R)) for q = 1 .. R-1.  FP64: one table entry,
      // then successive products (rounding grows by about one unit of 2^-53
      // per factor, and FP64 products cost four times FP32 ones, so fewer
      // table reads pay); FP32: every factor from the table
      const int kb = (t + TL * k) & (NS - 1);
      if constexpr (sizeof(v[0].x) == 8) {
        const T2 w1 = tw2(twl, kb * step);
        T2 w = w1;
#pragma unroll
        for (int q = 1; q < R; ++q) {
          v[k * R + q] = cmul(v[k * R + q], w);
          if (q + 1 < R) w = cmul(w, w1);
        }
      } else {
#pragma unroll
        for (int q = 1; q < R; ++q) v[k * R + q] = cmul(v[k * R + q], tw2(twl, q * kb * step));
      }
    }
    dft<R>(&v[k * R]);
  }
}

// Exchange after stage S: every output to its position of the line (LDS),
// then the inputs of stage S + 1 back into registers.  HALVES moves the real
// parts, then the imaginary parts, through a line of Reals.
template <int L, int S, bool HALVES, typename T2, typename Lds>
__device__ __forceinline__ void f2_exchange(T2 (&v)[16], int t, Lds* line) {
  constexpr int R = fft2::radix(L, S), NB = 16 / R, TL = fft2::threads(L);
  constexpr int R2 = fft2::radix(L, S + 1), NB2 = 16 / R2;
  if constexpr (HALVES) {
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
      for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int p = fft2::out_pos(L, S, t + TL * k, q);
          line[fft2::pad(p)] = part ? v[k * R + q].y : v[k * R + q].x;
        }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NB2; ++k)
#pragma unroll
        for (int q = 0; q < R2; ++q) {
          const int p = fft2::in_pos(L, S + 1, t + TL * k, q);
          if (part) v[k * R2 + q].y = line[fft2::pad(p)];
          else v[k * R2 + q].x = line[fft2::pad(p)];
        }
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
      for (int q = 0; q < R; ++q) line[fft2::pad(fft2::out_pos(L, S, t + TL * k, q))] = v[k * R + q];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NB2; ++k)
#pragma unroll
      for (int q = 0; q < R2; ++q) v[k * R2 + q] = line[fft2::pad(fft2::in_pos(L, S + 1, t + TL * k, q))];
    __syncthreads();
  }
}

// All stages of a line held by threads t of the workgroup (every thread of
// the workgroup calls this: the exchanges contain barriers).
template <int L, bool HALVES, typename T2, typename Lds>
__device__ __forceinline__ void f2_line(T2 (&v)[16], int t, Lds* line, const T2* twl) {
  f2_stage<L, 0>(v, t, twl);
  f2_exchange<L, 0, HALVES>(v, t, line);
  f2_stage<L, 1>(v, t, twl);
  if constexpr (fft2::nstages(L) > 2) {
    f2_exchange<L, 1, HALVES>(v, t, line);
    f2_stage<L, 2>(v, t, twl);
  }
  if constexpr (fft2::nstages(L) > 3) {
    f2_exchange<L, 2, HALVES>(v, t, line);
    f2_stage<L, 3>(v, t, twl);
  }
}

// register holding output index t + (L/16) j after the last stage
template <int L>
__device__ __forceinline__ constexpr int f2_reg_of(int j) {
  constexpr int R = fft2::radix(L, fft2::nstages(L) - 1), NB = 16 / R;
  return (j % NB) * R + j / NB;
}

// Arguments of the two-pass transform of one call.
template <typename Real>
struct Fft2Bufs {
  typename cplx<Real>::T* grid[3];  // natural layout [L0][L1]
  typename cplx<Real>::T* mid[3];   // first-pass result [L0][L1] (a buffer of its own)
  const unsigned char* rowflag[3];  // active rows of each grid's geometry
};

// LDS bytes of a first-pass workgroup: the exchange lines and the twiddle
// table of L0.
template <typename Real>
__host__ __device__ constexpr size_t f2_first_lds(int L0, int C, bool halves) {
  return (size_t)C * fft2::line_pitch_c(L0, C) * (halves ? sizeof(Real) : 2 * sizeof(Real)) +
         (size_t)tw2_count(L0) * 2 * sizeof(Real);
}
// LDS bytes of a last-pass workgroup: the exchange lines (reused for the
// grids' results) and the twiddle table of L1.
// The results of the G grids (all outputs, or half of them at a time with
// halves) are gathered in LDS for the power.
template <typename Real>
__host__ __device__ constexpr size_t f2_last_lds(int L1, int G, bool halves) {
  const size_t ex = (size_t)G * fft2::line_pitch(L1) * (halves ? sizeof(Real) : 2 * sizeof(Real));
  const size_t comb = G > 1 ? (size_t)G * (halves ? L1 / 2 : L1) * 2 * sizeof(Real) : 0;
  return (ex > comb ? ex : comb) + (size_t)tw2_count(L1) * 2 * sizeof(Real);
}

// LDS bytes of a last-pass workgroup that transforms the three grids of a
// row one after another: one exchange line and the twiddle table of L1.
template <typename Real>
__host__ __device__ constexpr size_t f2_last_seq_lds(int L1, bool halves) {
  return (size_t)fft2::line_pitch(L1) * (halves ? sizeof(Real) : 2 * sizeof(Real)) +
         (size_t)tw2_count(L1) * 2 * sizeof(Real);
}

}  // namespace mils
