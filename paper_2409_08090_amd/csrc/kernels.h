// kernels.h -- host-side launchers of the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "mils_internal.h"

namespace mils {

// Stages of the single-series path, for per-stage event timing.
enum Stage {
  kStageStats = 0,
  kStageBin = 1,
  kStageSpreadF = 2,
  kStageSpread2F = 3,
  kStagePass0 = 4,  // first FFT pass (pruned), then 5, 6 for later middle passes
  kStageLast = 7,   // last FFT pass + deconvolution + power
  kStageLow = 8,    // direct sums near f = 0
  kStageRows = 9,   // row classes of both geometries (two-pass plans)
  kStageOut = 10,   // transpose into frequency order (two-pass plans)
  kNumStages = 11
};

// A second stream for the 2f geometry of a periodogram, with the events
// that fork it from and join it back to the call's stream.
struct AuxStream {
  hipStream_t s;
  hipEvent_t fork, join;
  hipEvent_t mid;  // two-pass plans: the second branch's spread is done
};

// Optional hook called before (begin = 1) and after (begin = 0) each stage is
// enqueued; used to record HIP events around the stage's kernels.
struct StageHook {
  void (*fn)(void* ud, int stage, int begin, hipStream_t s);
  void* ud;
};

// Enqueue the whole single-series path (statistics, binning, spread, FFT
// passes, deconvolution and power or raw sums) on stream s.
hipError_t launch_path(const CallArgs& a, const Plan& p, const Work& w, hipStream_t s,
                       const StageHook* hook = nullptr, const AuxStream* aux = nullptr);

// 1 / phihat(m) for m = 0..K by Gauss-Legendre quadrature of the kernel.
// Series that share their observation times and weights: the weights-only
// call aw (y == NULL, unit_y set; statistics into w.stats) leaves the
// deconvolved sums B and B2 of every output frequency in bsum_b and bsum_b2
// (interleaved re/im), and the binning and row lists in w.
hipError_t launch_weight_sums(const CallArgs& aw, const Plan& p, const Work& w, double* bsum_b,
                              double* bsum_b2, hipStream_t s);

// Up to three such series at once: series g has values y[g], writes power[g]
// and keeps its statistics in stats[g] and its direct sums near f = 0 in
// lowfix[g]; its A sums go through grid g of the workspace.
struct SeriesGroup {
  int m;
  int need_sort;  // the weights-only call's sort decision (read back by the host)
  const double* y[3];
  double* power[3];
  DevStats* stats[3];
  double* lowfix[3];
};
// a: the call's arguments with bsum_b, bsum_b2 and wstats set; w: the
// workspace of the weights-only call (w.stats its statistics).
hipError_t launch_series_group(const CallArgs& a, const Plan& p, const Work& w,
                               const SeriesGroup& sg, hipStream_t s);

// Direct sums at every frequency, term by term, FP64 (statistics into
// w.stats, which with w.partials is all of w it uses): the power (a.power) or,
// with a.periodogram == 0, the raw sums of a.h (a.sums, interleaved re/im).
hipError_t launch_direct(const CallArgs& a, const Work& w, hipStream_t s);

// 1 / phihat in the order of the two-pass FFT's last pass (see k_phihat2).
hipError_t launch_phihat2(double* iphi2, const double* inv_phihat, int L0, int L1, int64_t n,
                          int64_t nf, int64_t K, hipStream_t s);

hipError_t launch_phihat(double* inv_phihat, int64_t K, double w, double n, const double* z,
                         const double* gphi, int q, hipStream_t s);

}  // namespace mils
