// batch.h -- descriptors of the persistent batched kernel (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mils_internal.h"

namespace mils {

// One series of a batch (device array, ordered by decreasing cost).
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

struct BatchArgs {
  const BatchCurve* curves;
  int ncurves;
  const Plan* plans;                 // per class
  const void* const* tw;             // per class twiddles
  const double* const* inv_phihat;   // per class kernel-transform table
  const double* t;
  const double* y;
  const double* dy;
  double* power;
  int norm, center, fit_mean;
  unsigned int* counter;             // work queue head (reset by the launch)
  int* status;                       // per series, caller order
  Work w0;                           // workspace of slot 0
  size_t slot_stride;                // bytes between slots
};

// Enqueue the counter reset and the persistent kernel (nslots workgroups).
hipError_t launch_batch(const BatchArgs& ba, int nslots, int prec, hipStream_t s);

}  // namespace mils
