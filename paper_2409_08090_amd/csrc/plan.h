// plan.h -- host-side planner: kernel width and shape from the tolerance,
// fine-grid size and its multi-pass FFT factorisation, twiddle tables and the
// quadrature nodes of the kernel's Fourier transform.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "mils_internal.h"

namespace mils {

struct PlanRequest {
  int64_t nf;
  double eps;
  int prec;             // 0 FP64, 1 FP32
  int G;                // grids transformed together in the last pass (3 or 1)
  double sigma = 0.0;   // upsampling factor; 0 = the precision's default
  bool batch = false;   // plan for the batched kernels (no big passes)
  int64_t n_fixed = 0;  // use exactly this grid size (must factor), 0 = choose
  int tile_max = 0;     // largest spreading tile (cells), 0 = kTileMax
  bool fft2 = false;    // the two-pass register-tile FFT may replace plans of 3+ passes
};

// Default upsampling factor of a precision (1.25 in both).
double default_sigma(int prec);

// Smallest upsampling factor the planner uses for a tolerance when none is
// requested (batch: a plan for the batched kernels).
double planner_sigma(double eps, int prec, bool batch);

// Kernel width for tolerance eps at upsampling sigma (clamped to [2, 20]).
int kernel_width(double eps, double sigma, int prec);

// Shape parameter of the exponential-of-semicircle kernel.
double kernel_beta(int w, double sigma);

// Build the plan; returns false (with a message) when no supported
// factorisation exists.
bool make_plan(const PlanRequest& r, Plan* out, std::string* err);

// Twiddle tables of the plan, as interleaved (re, im) pairs in FP64; the
// caller narrows them to FP32 for FP32 plans.  Offsets are stored in the plan.
void make_twiddles(Plan* p, std::vector<double>* tw);

// Gauss-Legendre nodes z_r in (0, 1) and the products g_r * phi(z_r) used by
// the phihat kernel (even rule of q points on [-1, 1], positive half).
void phihat_nodes(const Plan& p, std::vector<double>* z, std::vector<double>* gphi);

// Monomial coefficients of the kernel polynomials (Chebyshev interpolation of
// phi((k + t)/hw - 1), t in [0, 1], in long double): coef[j * kHornerK + k],
// j = 0 the highest degree, horner_n(p.prec) coefficients, k < kHornerK.
void make_horner(const Plan& p, std::vector<double>* coef);

// Device workspace layout of one call; returns the byte size.  With base ==
// nullptr only the size is computed.
// Workspace of one call (nd points, G grids) at base (nullptr: size only).
// per_series: the workspace of one series of a batch, without the buffers of
// the multi-workgroup reductions of the single-series path.
size_t layout_work(const Plan& p, int64_t nd, int G, char* base, Work* w,
                   bool per_series = false);

}  // namespace mils
