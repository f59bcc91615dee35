// batch.h -- descriptors of the batched periodogram kernels (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mils_internal.h"

namespace mils {

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
};

// A unit of work of a batched phase: series `curve` (index into curves),
// and `sub`: the spreading tile, g * nblk + blk for a first/middle FFT pass,
// or the row block of the last pass.
struct BatchItem {
  int curve;
  int sub;
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
  size_t pass_lds[kMaxPass - 1];     // dynamic LDS of each pass launch
  size_t last_lds;
};

// Enqueue the kernels of a batch: per-series statistics, binning and direct
// low-frequency sums; both spreads; the FFT passes; the last pass with power.
hipError_t launch_batch(const BatchLaunch& bl, hipStream_t s);

}  // namespace mils
