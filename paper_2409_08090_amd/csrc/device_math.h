// device_math.h -- double-double helpers, grid coordinates, the
// exponential-of-semicircle kernel and small complex arithmetic for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mils {

// ---- error-free transformations --------------------------------------------
__device__ __forceinline__ void dd_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// The rounded product passes through an empty asm statement: the compiler
// then cannot contract it into a later subtraction (p - floor(p) would
// become fma(a, b, -floor(p)), and adding e would count the product's
// rounding error twice).
__device__ __forceinline__ void dd_two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  asm("" : "+v"(p));
  e = __builtin_fma(a, b, -p);
}

// Grid coordinate of a point: u = n * frac(g * (t - tau)) split as
// cell (integer in [0, n)) + frac (in [0, 1)).  The shift t - tau, the product
// with the frequency step g and the scaling by n are carried in double-double,
// so u is the exact coordinate of the binary64 inputs to ~1e-16 of a cell.
__device__ __forceinline__ void grid_coord(double t, double tau, double g, double nd_,
                                           int64_t n, int64_t& cell, double& frac) {
  double th, tl;
  dd_two_sum(t, -tau, th, tl);
  double ph, pl;
  dd_two_prod(g, th, ph, pl);
  pl = __builtin_fma(g, tl, pl);
  double fh = ph - floor(ph);  // exact
  double uh, ul;
  dd_two_prod(nd_, fh, uh, ul);
  ul = __builtin_fma(nd_, pl, ul);
  double ci = floor(uh);
  double d = (uh - ci) + ul;
  double fl = floor(d);
  ci += fl;
  d -= fl;
  if (d >= 1.0) {
    d -= 1.0;
    ci += 1.0;
  }
  int64_t c = (int64_t)ci;
  c %= n;
  if (c < 0) c += n;
  cell = c;
  frac = d;
}

// The same with 32-bit cell indices (grids up to 2^31 cells).
__device__ __forceinline__ void grid_coord32(double t, double tau, double g, double nd_, int n,
                                             int& cell, double& frac) {
  double th, tl;
  dd_two_sum(t, -tau, th, tl);
  double ph, pl;
  dd_two_prod(g, th, ph, pl);
  pl = __builtin_fma(g, tl, pl);
  double fh = ph - floor(ph);  // exact
  double uh, ul;
  dd_two_prod(nd_, fh, uh, ul);
  ul = __builtin_fma(nd_, pl, ul);
  double ci = floor(uh);
  double d = (uh - ci) + ul;
  double fl = floor(d);
  ci += fl;
  d -= fl;
  if (d >= 1.0) {
    d -= 1.0;
    ci += 1.0;
  }
  int c = (int)ci;
  if (c >= n) c -= n;
  if (c < 0) c += n;
  cell = c;
  frac = d;
}

// exp(+2 pi i f_c (t - tau)) with the phase reduced in double-double.
__device__ __forceinline__ void prephase(double t, double tau, double fch, double fcl,
                                         double& c, double& s) {
  double th, tl;
  dd_two_sum(t, -tau, th, tl);
  double ah, al;
  dd_two_prod(fch, th, ah, al);
  al = __builtin_fma(fch, tl, al);
  al = __builtin_fma(fcl, th, al);
  double r = (ah - floor(ah)) + al;
  r -= rint(r);
  sincospi(2.0 * r, &s, &c);
}

// Exponential-of-semicircle kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| <= 1.
__device__ __forceinline__ double es_kernel(double z, double beta) {
  double a = 1.0 - z * z;
  return a >= 0.0 ? exp(beta * (sqrt(a) - 1.0)) : 0.0;
}
__device__ __forceinline__ float es_kernel(float z, float beta) {
  float a = 1.0f - z * z;
  return a >= 0.0f ? __expf(beta * (__fsqrt_rn(a) - 1.0f)) : 0.0f;
}

// ---- complex helpers --------------------------------------------------------
template <typename R>
struct cplx;
template <>
struct cplx<double> {
  using T = double2;
};
template <>
struct cplx<float> {
  using T = float2;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// Streaming (nontemporal) loads and stores, for data read or written once:
// marked so that the caches do not keep them in place of data that is used
// again.
typedef double d2v_t __attribute__((ext_vector_type(2)));
typedef float f2v_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const d2v_t w = __builtin_nontemporal_load(reinterpret_cast<const d2v_t*>(p));
  return make_double2(w.x, w.y);
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const f2v_t w = __builtin_nontemporal_load(reinterpret_cast<const f2v_t*>(p));
  return make_float2(w.x, w.y);
}
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
  const d2v_t w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<d2v_t*>(p));
}
__device__ __forceinline__ void st_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by +i
__device__ __forceinline__ double2 cmuli(double2 a) { return make_double2(-a.y, a.x); }
__device__ __forceinline__ float2 cmuli(float2 a) { return make_float2(-a.y, a.x); }
template <typename T2, typename R>
__device__ __forceinline__ T2 cscale(T2 a, R s) {
  T2 r;
  r.x = a.x * s;
  r.y = a.y * s;
  return r;
}
template <typename T2>
__device__ __forceinline__ T2 czero() {
  T2 r;
  r.x = 0;
  r.y = 0;
  return r;
}

// XCD-aware block remap: hardware dispatches consecutive workgroups round-robin
// over the 8 XCDs; this maps them so that each XCD receives a contiguous range
// of logical blocks (neighbouring tiles share that XCD's L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t nx = 8;
  if (nblocks < nx) return bid;
  int64_t per = nblocks / nx;
  int64_t rem = nblocks - per * nx;
  int64_t x = bid % nx;
  int64_t i = bid / nx;
  // blocks beyond per*nx on XCD x: those with i == per (only for x < rem)
  int64_t start = x * per + (x < rem ? x : rem);
  return start + i;
}

}  // namespace mils
