// batch.h -- descriptors of the batched periodogram kernels (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mils_internal.h"

namespace mils {

// Series whose three grids fit one workgroup's LDS run the whole pipeline in
// that workgroup (k_bsmall): the grids are FP64 complex, interleaved
// (element l of grid g at 3 l + g), next to the two-level twiddle table of n.
// The radix stages of the in-LDS transform keep every butterfly index below
// 2048 and every stage's Ns at most 1024 (the exact float division of the
// Stockham stage), hence n <= kSmallMaxN and a last radix with n / R <= 1024.
constexpr int kSmallMaxN = 3072;
constexpr int kSmallMaxRad = 12;
constexpr size_t kSmallLdsCap = 147 * 1024;  // dynamic LDS beside the kernel's static 13 KB (160 KB per CU)
__host__ __device__ constexpr inline size_t small_lds_bytes(int64_t n) {
  return (size_t)(48 * n + 16 * (64 + (n + 63) / 64));
}

// One series of a batch (device array).
struct BatchCurve {
  int64_t t_off;    // first point in t, y, dy
  int64_t nd;       // points
  int64_t out_off;  // first output in power
  int64_t nf;       // frequencies of this series
  int64_t K;        // floor(nf / 2)
  double f0, df;
  double fch, fcl;  // f0 + K df as a double-double
  int64_t kzero;    // output index of the zero frequency, or -1
  int plan;         // grid-size class (index into the plan arrays)
  int index;        // position of the series in the caller's order
  int small;        // 1: the whole pipeline in one workgroup's LDS (k_bsmall)
  int nsrad;        // radix stages of the in-LDS transform of the n-cell grid
  signed char srad[kSmallMaxRad];
};

// A unit of work of a batched phase: series `curve` (index into curves),
// and `sub`: the spreading tile, the column block of a first/middle FFT pass
// (FP64: all three grids; FP32: g * nblk + blk for grid g), or the row block
// of the last pass.
struct BatchItem {
  int curve;
  int sub;
  int plan;  // the series' grid-size class (a copy of curves[curve].plan, so
             // that the plan's parameters load beside the series' descriptors)
};

struct BatchArgs {
  const BatchCurve* curves;
  int ncurves;
  const Plan* plans;                 // per class
  const void* const* tw;             // per class twiddles
  const double* const* inv_phihat;   // per class kernel-transform table
  const Work* works;                 // per series workspace
  const double* t;
  const double* y;
  const double* dy;
  double* power;
  int norm, center, fit_mean;
  double dmin;  // power NaN where the fit's determinant is at most dmin
  int* status;                       // per series, caller order
};

// Grids per workgroup of a batched first/middle FFT pass: all three in FP64,
// one in FP32 (its items are then g * nblk + blk).
template <typename Real>
constexpr int kBatchPassGrids = sizeof(Real) == 8 ? 3 : 1;

// The launches of one batch (or of one chunk of it), in order.
struct BatchLaunch {
  BatchArgs args;
  int prec;
  const BatchItem* spread_items;     // every tile of every series (both geometries use them)
  int nspread;
  const BatchItem* pass_items[kMaxPass - 1];  // first/middle pass ip
  int npass_items[kMaxPass - 1];
  const BatchItem* last_items;
  int nlast;
  const BatchItem* small_items;      // series that run entirely in LDS
  int nsmall;
  size_t small_lds;                  // dynamic LDS of that launch (largest grid)
  size_t pass_lds[kMaxPass - 1];     // dynamic LDS of each pass launch
  size_t last_lds;
};

// Enqueue the kernels of a batch: the series that fit LDS in one launch; for
// the others per-series statistics, binning and direct low-frequency sums,
// both spreads, the FFT passes, the last pass with power.
hipError_t launch_batch(const BatchLaunch& bl, hipStream_t s);

// Allows the on-chip kernel its dynamic LDS (before any launch or capture).
hipError_t batch_prepare();

}  // namespace mils
