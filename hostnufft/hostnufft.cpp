// hostnufft.cpp -- a plain host FP64 NUFFT Lomb-Scargle periodogram.
//
// CPU BASELINE FOR TIMING ONLY.  Nothing in the GPU library calls, links or
// includes this file, and it uses nothing from the library or from the
// oracle.  The benchmark times it beside the GPU path on the same inputs, on
// every host core, as the stand-in for the CPU backend of the paper (Sec. 2,
// Sec. 2.1: the type-1 NUFFT evaluated on the CPU).
//
// What it computes (nifty-ls paper, Sec. 1, Eq. 1 and Eq. 2): the sums
// sum_j h_j exp(+2 pi i f_k t_j) on f_k = f0 + k df as a type-1 NUFFT --
// spread the phase-shifted strengths onto an upsampled periodic grid with the
// exponential-of-semicircle kernel, FFT, divide by the kernel's Fourier
// transform -- for the three sums of a floating-mean periodogram (data and
// weights at f, weights at 2f), then the least-squares power per frequency.
//
// Choices (all of this file's own):
//   - upsampling sigma = 2 and width w = ceil(log10(1/eps)) + 2, beta = 2.30 w
//     (the published sigma = 2 rule of the exponential-of-semicircle papers
//     the method cites, with one cell of margin);
//   - grid n = smallest 2^a 3^b 5^c >= 2 nf, modes m = k - floor(nf/2);
//   - phases f t and grid coordinates df t reduced modulo one in
//     double-double, no time shift;
//   - spreading by cell blocks: each block gathers the points whose kernel
//     reaches it (points ordered by grid coordinate), so every cell is written
//     by one thread;
//   - the FFT is a four-step transform (n = n1 n2) of iterative Stockham
//     radix-4/2/3/5 sub-transforms, OpenMP over columns and rows;
//   - the kernel transform by Gauss-Legendre quadrature;
//   - the frequencies with |f| span < 2 (at most 16 nearest f = 0) by direct
//     double-double sums, since the floating-mean terms cancel there.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;
constexpr double kTwoPi = 6.283185307179586476925286766559;

// ---- double-double helpers ----------------------------------------------
inline void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = std::fma(a, b, -p);
}
inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
// frac(x) of the double-double (hi, lo), in [0, 1)
inline double dd_frac(double hi, double lo) {
  const double fh = hi - std::floor(hi);  // exact
  double s = fh + lo;
  s -= std::floor(s);
  if (s >= 1.0) s -= 1.0;
  return s;
}
// frac((a_hi + a_lo) * t)
inline double frac_prod(double a_hi, double a_lo, double t) {
  double p, e;
  two_prod(a_hi, t, p, e);
  return dd_frac(p, e + a_lo * t);
}

// ---- FFT: iterative Stockham, sign +, unnormalised -----------------------
struct SubFft {
  int64_t n = 0;
  std::vector<int> radix;
  std::vector<cplx> root;  // exp(+2 pi i x / n), x < n
};

void make_subfft(SubFft& f, int64_t n) {
  f.n = n;
  f.radix.clear();
  int64_t m = n;
  while (m % 4 == 0) { f.radix.push_back(4); m /= 4; }
  while (m % 2 == 0) { f.radix.push_back(2); m /= 2; }
  while (m % 3 == 0) { f.radix.push_back(3); m /= 3; }
  while (m % 5 == 0) { f.radix.push_back(5); m /= 5; }
  f.root.resize(n);
  for (int64_t x = 0; x < n; ++x) {
    const long double a = 2.0L * 3.14159265358979323846264338327950288L * x / n;
    f.root[x] = cplx((double)std::cos(a), (double)std::sin(a));
  }
}

// Transform x (length f.n) using scratch y of the same length; the result
// ends in x.
void subfft(const SubFft& f, cplx* x, cplx* y) {
  const int64_t n = f.n;
  cplx* in = x;
  cplx* out = y;
  int64_t ns = 1;  // length of the transforms already done
  for (int R : f.radix) {
    const int64_t nb = n / R;
    const int64_t tstep = n / (ns * R);
    for (int64_t j = 0; j < nb; ++j) {
      const int64_t k = j % ns;
      cplx v[5];
      for (int r = 0; r < R; ++r) v[r] = in[j + r * nb];
      if (ns > 1)
        for (int r = 1; r < R; ++r) v[r] *= f.root[(r * k * tstep) % n];
      cplx o[5];
      if (R == 2) {
        o[0] = v[0] + v[1];
        o[1] = v[0] - v[1];
      } else if (R == 4) {
        const cplx a = v[0] + v[2], b = v[0] - v[2];
        const cplx c = v[1] + v[3];
        const cplx d = (v[1] - v[3]) * cplx(0.0, 1.0);
        o[0] = a + c;
        o[2] = a - c;
        o[1] = b + d;
        o[3] = b - d;
      } else if (R == 3) {
        const double s3 = 0.86602540378443864676;
        const cplx a = v[1] + v[2];
        const cplx d = (v[1] - v[2]) * cplx(0.0, s3);
        const cplx m = v[0] - 0.5 * a;
        o[0] = v[0] + a;
        o[1] = m + d;
        o[2] = m - d;
      } else {  // 5, from the definition with exp(+2 pi i r q / 5)
        for (int q = 0; q < 5; ++q) {
          cplx acc = v[0];
          for (int r = 1; r < 5; ++r) acc += v[r] * f.root[((int64_t)r * q % 5) * (n / 5)];
          o[q] = acc;
        }
      }
      const int64_t base = (j / ns) * ns * R + k;
      for (int r = 0; r < R; ++r) out[base + r * ns] = o[r];
    }
    std::swap(in, out);
    ns *= R;
  }
  if (in != x) std::memcpy(x, in, sizeof(cplx) * n);
}

// Four-step transform of length n = n1 n2 (x viewed as [n1][n2], element
// l = l1 n2 + l2): column transforms over l1, twiddle exp(2 pi i l2 m1 / n),
// row transforms over l2; output mode m = m1 + n1 m2 is left at x[m1 n2 + m2].
struct BigFft {
  int64_t n = 0, n1 = 0, n2 = 0;
  SubFft c, r;
  int bsh = 0;
  std::vector<cplx> lo, hi;  // exp(2 pi i x / n) = lo[x & mask] * hi[x >> bsh]
  cplx tw(int64_t x) const {
    return lo[x & (((int64_t)1 << bsh) - 1)] * hi[x >> bsh];
  }
};

void make_bigfft(BigFft& b, int64_t n) {
  b.n = n;
  // n1: the divisor of n closest to sqrt(n) from below
  int64_t best = 1;
  for (int64_t d = 1; d * d <= n; ++d)
    if (n % d == 0) best = d;
  b.n1 = best;
  b.n2 = n / best;
  make_subfft(b.c, b.n1);
  make_subfft(b.r, b.n2);
  b.bsh = 0;
  while (((int64_t)1 << (2 * b.bsh)) < n) ++b.bsh;
  const int64_t B = (int64_t)1 << b.bsh;
  const long double pi2 = 2.0L * 3.14159265358979323846264338327950288L;
  b.lo.resize(B);
  for (int64_t x = 0; x < B; ++x) {
    const long double a = pi2 * x / n;
    b.lo[x] = cplx((double)std::cos(a), (double)std::sin(a));
  }
  b.hi.resize(n / B + 1);
  for (int64_t x = 0; x <= n / B; ++x) {
    const long double a = pi2 * (long double)((x * B) % n) / n;
    b.hi[x] = cplx((double)std::cos(a), (double)std::sin(a));
  }
}

// x: n values; scratch: n values.  Threads: the OpenMP team of the caller
// (nested levels off).
void bigfft(const BigFft& b, cplx* x, cplx* scratch, int nthreads) {
  const int64_t n1 = b.n1, n2 = b.n2;
  constexpr int64_t kCols = 8;  // columns gathered together (cache lines)
  // columns: gather kCols columns, transform, twiddle, scatter back
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (int64_t c0 = 0; c0 < n2; c0 += kCols) {
    const int64_t nc = std::min(kCols, n2 - c0);
    std::vector<cplx> col((size_t)kCols * n1), tmp(n1);
    for (int64_t l1 = 0; l1 < n1; ++l1)
      for (int64_t q = 0; q < nc; ++q) col[q * n1 + l1] = x[l1 * n2 + c0 + q];
    for (int64_t q = 0; q < nc; ++q) {
      subfft(b.c, col.data() + q * n1, tmp.data());
      const int64_t l2 = c0 + q;
      for (int64_t m1 = 0; m1 < n1; ++m1) col[q * n1 + m1] *= b.tw((l2 * m1) % b.n);
    }
    for (int64_t m1 = 0; m1 < n1; ++m1)
      for (int64_t q = 0; q < nc; ++q) x[m1 * n2 + c0 + q] = col[q * n1 + m1];
  }
  (void)scratch;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
  for (int64_t m1 = 0; m1 < n1; ++m1) {
    std::vector<cplx> tmp(n2);
    subfft(b.r, x + m1 * n2, tmp.data());
  }
}

// mode m of a four-step output
inline const cplx& mode_at(const BigFft& b, const cplx* x, int64_t m) {
  const int64_t m1 = m % b.n1, m2 = m / b.n1;
  return x[m1 * b.n2 + m2];
}

// ---- Plan ------------------------------------------------------------------
bool smooth235(int64_t x) {
  for (int f : {2, 3, 5})
    while (x % f == 0) x /= f;
  return x == 1;
}

struct Plan {
  int64_t n;
  int w;
  double beta;
  BigFft fft;
  std::vector<double> phihat;  // phihat(m), m = 0 .. n/2
};

// Gauss-Legendre nodes and weights on [0, 1] (q points) by Newton iteration
// on the Legendre polynomial P_q.
void gauss_legendre01(int q, std::vector<double>& x, std::vector<double>& wt) {
  x.resize(q);
  wt.resize(q);
  for (int i = 0; i < q; ++i) {
    long double z = std::cos(3.14159265358979323846L * (i + 0.75L) / (q + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1);
      const long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    // node z in [-1, 1] -> (z + 1) / 2 in [0, 1]
    x[i] = (double)((z + 1) / 2);
    wt[i] = (double)(1.0L / ((1 - z * z) * dp * dp));  // weight on [0, 1]
  }
}

int64_t grid_size(int64_t nf) {
  int64_t n = 2 * nf;
  if (n < 16) n = 16;
  while (!smooth235(n)) ++n;
  return n;
}

std::unique_ptr<Plan> make_plan(int64_t n, double eps) {
  auto p = std::make_unique<Plan>();
  p->n = n;
  int w = (int)std::ceil(std::log10(1.0 / eps)) + 2;
  w = std::max(4, std::min(w, 18));
  p->w = w;
  p->beta = 2.30 * w;
  make_bigfft(p->fft, n);
  // phihat(m) = int phi(z / (w/2)) exp(2 pi i m z / n) dz over |z| < w/2
  //           = w * int_0^1 phi(s) cos(pi m w s / n) ds,  phi(s) = exp(beta (sqrt(1 - s^2) - 1))
  std::vector<double> xs, ws;
  gauss_legendre01(3 * w + 20, xs, ws);
  std::vector<double> g(xs.size());
  for (size_t i = 0; i < xs.size(); ++i)
    g[i] = ws[i] * std::exp(p->beta * (std::sqrt(1.0 - xs[i] * xs[i]) - 1.0));
  const int64_t K = n / 2;
  p->phihat.resize(K + 1);
  const double pi = kTwoPi / 2;
#pragma omp parallel for schedule(static)
  for (int64_t m = 0; m <= K; ++m) {
    double acc = 0.0;
    for (size_t i = 0; i < xs.size(); ++i) acc += g[i] * std::cos(pi * m * w * xs[i] / n);
    p->phihat[m] = w * acc;
  }
  return p;
}

std::mutex g_plan_mu;
std::map<std::pair<int64_t, double>, std::unique_ptr<Plan>> g_plans;

// Plans are kept per grid size (the kernel transform table covers every mode
// of the grid, so all frequency counts with the same grid share one).
const Plan* get_plan(int64_t nf, double eps) {
  const int64_t n = grid_size(nf);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto key = std::make_pair(n, eps);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) return it->second.get();
  auto p = make_plan(n, eps);
  const Plan* r = p.get();
  g_plans[key] = std::move(p);
  return r;
}

// ---- spreading -------------------------------------------------------------
// Points of one geometry in the order of their grid coordinate u in [0, n).
struct Geometry {
  std::vector<double> u;      // sorted coordinates
  std::vector<int64_t> idx;   // point index of each
};

void order_points(const std::vector<double>& u_by_point, Geometry& g) {
  const int64_t nd = (int64_t)u_by_point.size();
  g.idx.resize(nd);
  // a rotation of a sorted sequence needs no sort (sorted times, span < 1/df)
  int64_t drops = 0, start = 0;
  for (int64_t j = 1; j < nd; ++j)
    if (u_by_point[j] < u_by_point[j - 1]) {
      ++drops;
      start = j;
    }
  if (drops == 0 || (drops == 1 && u_by_point[nd - 1] <= u_by_point[0])) {
    for (int64_t j = 0; j < nd; ++j) g.idx[j] = (start + j) % nd;
  } else {
    for (int64_t j = 0; j < nd; ++j) g.idx[j] = j;
    std::sort(g.idx.begin(), g.idx.end(),
              [&](int64_t a, int64_t b) { return u_by_point[a] < u_by_point[b]; });
  }
  g.u.resize(nd);
  for (int64_t j = 0; j < nd; ++j) g.u[j] = u_by_point[g.idx[j]];
}

// Spread NG strength vectors (complex, by point) of one geometry onto NG grids
// of n cells: grid[l] = sum_j h_j phi((l - u_j) / (w/2)) over the periodic
// images, parallel over blocks of cells.
void spread(const Plan& p, const Geometry& g, int NG, const cplx* const* h, cplx* const* grid,
            int nthreads) {
  const int64_t n = p.n, nd = (int64_t)g.u.size();
  const double hw = 0.5 * p.w;
  constexpr int64_t kBlock = 4096;
  const int64_t nblk = (n + kBlock - 1) / kBlock;
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t c0 = b * kBlock, c1 = std::min(n, c0 + kBlock);
    for (int q = 0; q < NG; ++q) std::fill(grid[q] + c0, grid[q] + c1, cplx(0.0, 0.0));
    // points with u in [c0 - hw, c1 + hw), cyclically: up to three windows
    const double lo = c0 - hw, hi = c1 + hw;
    const double wins[3][2] = {{lo, hi}, {lo + n, hi + n}, {lo - n, hi - n}};
    for (const auto& wv : wins) {
      const double a = std::max(wv[0], 0.0), e = std::min(wv[1], (double)n);
      if (a >= e) continue;
      const double shift = wv[0] - lo;  // n, 0 or -n: the image of the points
      const int64_t j0 = std::lower_bound(g.u.begin(), g.u.end(), a) - g.u.begin();
      const int64_t j1 = std::lower_bound(g.u.begin(), g.u.end(), e) - g.u.begin();
      for (int64_t j = j0; j < j1; ++j) {
        const double u = g.u[j] - shift;  // coordinate relative to this block's frame
        const int64_t lfirst = std::max<int64_t>(c0, (int64_t)std::ceil(u - hw));
        const int64_t llast = std::min<int64_t>(c1 - 1, (int64_t)std::floor(u + hw));
        const int64_t pj = g.idx[j];
        for (int64_t l = lfirst; l <= llast; ++l) {
          const double z = (l - u) / hw;
          const double a2 = 1.0 - z * z;
          if (a2 <= 0.0) continue;
          const double phi = std::exp(p.beta * (std::sqrt(a2) - 1.0));
          for (int q = 0; q < NG; ++q) grid[q][l] += phi * h[q][pj];
        }
      }
    }
    (void)nd;
  }
}

// ---- power -----------------------------------------------------------------
double ls_power(cplx A, cplx B, cplx B2, double Ybar, double YY, double W, int norm,
                int fit_mean) {
  // sums of w^ cos^2, sin^2, cos sin from the double-angle sums
  double cc = 0.5 * (1.0 + B2.real()), ss = 0.5 * (1.0 - B2.real()), cs = 0.5 * B2.imag();
  double yc = A.real(), ys = A.imag();
  if (fit_mean) {
    cc -= B.real() * B.real();
    ss -= B.imag() * B.imag();
    cs -= B.real() * B.imag();
    yc -= Ybar * B.real();
    ys -= Ybar * B.imag();
  }
  const double det = cc * ss - cs * cs;
  if (!(det > 0.0)) return std::nan("");
  const double num = ss * yc * yc + cc * ys * ys - 2.0 * cs * yc * ys;
  switch (norm) {
    case 1: return num / (YY * det - num);
    case 2: return -std::log1p(-num / (YY * det));
    case 3: return 0.5 * W * num / det;
    default: return num / (YY * det);
  }
}

struct Work {
  std::vector<cplx> g[3];
  std::vector<cplx> scratch;
};

// One periodogram; nthreads for every parallel loop.
int periodogram(const double* t, const double* y, const double* dy, int64_t nd, double f0,
                double df, int64_t nf, double eps, int norm, int center, int fit_mean,
                int nthreads, double* power, Work& wk) {
  if (nd < 1 || nf < 1 || !(df > 0.0)) return -1;
  const Plan& p = *get_plan(nf, eps);
  const int64_t n = p.n, K = nf / 2;
  // weights and moments
  std::vector<double> wv(nd);
  double W = 0.0;
  for (int64_t j = 0; j < nd; ++j) {
    wv[j] = dy ? 1.0 / (dy[j] * dy[j]) : 1.0;
    W += wv[j];
  }
  double ybar = 0.0;
  for (int64_t j = 0; j < nd; ++j) ybar += wv[j] * y[j];
  ybar /= W;
  const double ysub = center ? ybar : 0.0;
  double Ybar = 0.0, yy = 0.0;
  for (int64_t j = 0; j < nd; ++j) {
    const double d = y[j] - ysub;
    Ybar += wv[j] * d;
    yy += wv[j] * d * d;
  }
  Ybar /= W;
  yy /= W;
  const double YY = fit_mean ? yy - Ybar * Ybar : yy;
  if (!(YY > 0.0)) return -2;
  double tmin = t[0], tmax = t[0];
  for (int64_t j = 1; j < nd; ++j) {
    tmin = std::min(tmin, t[j]);
    tmax = std::max(tmax, t[j]);
  }
  // centre frequency f_c = f0 + K df as a double-double, and 2 f_c, 2 df
  double kp, ke, fch, fcl;
  two_prod((double)K, df, kp, ke);
  two_sum(f0, kp, fch, fcl);
  fcl += ke;
  // per point: coordinates and strengths of both geometries
  std::vector<double> u1(nd), u2(nd);
  std::vector<cplx> hA(nd), hB(nd), hB2(nd);
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t j = 0; j < nd; ++j) {
    const double x1 = frac_prod(df, 0.0, t[j]);
    const double x2 = frac_prod(2.0 * df, 0.0, t[j]);
    u1[j] = std::min(x1 * n, std::nextafter((double)n, 0.0));
    u2[j] = std::min(x2 * n, std::nextafter((double)n, 0.0));
    const double ph = frac_prod(fch, fcl, t[j]);
    const cplx e(std::cos(kTwoPi * ph), std::sin(kTwoPi * ph));
    const double wh = wv[j] / W;
    hA[j] = (wh * (y[j] - ysub)) * e;
    hB[j] = wh * e;
    hB2[j] = wh * (e * e);
  }
  Geometry g1, g2;
  order_points(u1, g1);
  order_points(u2, g2);
  for (int q = 0; q < 3; ++q) wk.g[q].resize(n);
  wk.scratch.resize(1);
  {
    const cplx* h1[2] = {hA.data(), hB.data()};
    cplx* o1[2] = {wk.g[0].data(), wk.g[1].data()};
    spread(p, g1, 2, h1, o1, nthreads);
    const cplx* h2[1] = {hB2.data()};
    cplx* o2[1] = {wk.g[2].data()};
    spread(p, g2, 1, h2, o2, nthreads);
  }
  for (int q = 0; q < 3; ++q) bigfft(p.fft, wk.g[q].data(), wk.scratch.data(), nthreads);
  // direct sums near f = 0
  const double span = tmax - tmin;
  std::vector<int64_t> lowk;
  if (span > 0.0) {
    const double fl = 2.0 / span;
    const double ka = std::max(0.0, std::ceil((-fl - f0) / df));
    const double kb = std::min((double)(nf - 1), std::floor((fl - f0) / df));
    if (kb >= ka) {
      double lo = ka;
      if (kb - ka + 1 > 16) {
        lo = std::rint(-f0 / df) - 8;
        lo = std::max(ka, std::min(lo, kb - 15));
      }
      for (double k = lo; k <= kb && lowk.size() < 16; k += 1.0) lowk.push_back((int64_t)k);
    }
  }
  std::vector<cplx> lowA(lowk.size()), lowB(lowk.size()), lowB2(lowk.size());
  for (size_t i = 0; i < lowk.size(); ++i) {
    double fp, fe, fh, fl2;
    two_prod((double)lowk[i], df, fp, fe);
    two_sum(f0, fp, fh, fl2);
    fl2 += fe;
    cplx a(0, 0), b(0, 0), b2(0, 0);
    for (int64_t j = 0; j < nd; ++j) {
      const double ph = frac_prod(fh, fl2, t[j]);
      const cplx e(std::cos(kTwoPi * ph), std::sin(kTwoPi * ph));
      const double wh = wv[j] / W;
      a += (wh * (y[j] - ysub)) * e;
      b += wh * e;
      b2 += wh * (e * e);
    }
    lowA[i] = a;
    lowB[i] = b;
    lowB2[i] = b2;
  }
  // deconvolution, crop and power
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t k = 0; k < nf; ++k) {
    const int64_t m = k - K;
    const int64_t mm = m < 0 ? m + n : m;
    const double ip = 1.0 / p.phihat[m < 0 ? -m : m];
    cplx A = mode_at(p.fft, wk.g[0].data(), mm) * ip;
    cplx B = mode_at(p.fft, wk.g[1].data(), mm) * ip;
    cplx B2 = mode_at(p.fft, wk.g[2].data(), mm) * ip;
    for (size_t i = 0; i < lowk.size(); ++i)
      if (lowk[i] == k) {
        A = lowA[i];
        B = lowB[i];
        B2 = lowB2[i];
      }
    double pw = ls_power(A, B, B2, Ybar, YY, W, norm, fit_mean);
    // f == 0 exactly: defined as zero power
    if (f0 + (double)k * df == 0.0) pw = 0.0;
    power[k] = pw;
  }
  return 0;
}

}  // namespace

extern "C" {

int hostnufft_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Build (and cache) the plan of nf frequencies at tolerance eps; returns the
// grid size n.
int64_t hostnufft_plan(int64_t nf, double eps) { return get_plan(nf, eps)->n; }

// One periodogram (power[nf], host arrays).  norm: 0 standard, 1 model,
// 2 log, 3 psd.  Returns 0, -1 (invalid arguments) or -2 (constant data).
int hostnufft_periodogram(const double* t, const double* y, const double* dy, int64_t nd,
                          double f0, double df, int64_t nf, double eps, int norm, int center,
                          int fit_mean, int nthreads, double* power) {
  Work wk;
  return periodogram(t, y, dy, nd, f0, df, nf, eps, norm, center, fit_mean, nthreads, power, wk);
}

// Many series in CSR layout (nd_off, nf_off: ncurves + 1 offsets), one
// series per thread at a time; status[i] as for one periodogram.
int hostnufft_batch(int64_t ncurves, const int64_t* nd_off, const double* t, const double* y,
                    const double* dy, const int64_t* nf_off, const double* f0, const double* df,
                    double eps, int norm, int center, int fit_mean, int nthreads, double* power,
                    int32_t* status) {
  int bad = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : bad)
  {
    Work wk;
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < ncurves; ++i) {
      const int64_t a = nd_off[i], nd = nd_off[i + 1] - a;
      const int64_t b = nf_off[i], nf = nf_off[i + 1] - b;
      const int rc = periodogram(t + a, y + a, dy ? dy + a : nullptr, nd, f0[i], df[i], nf, eps,
                                 norm, center, fit_mean, 1, power + b, wk);
      if (status) status[i] = rc;
      if (rc) ++bad;
    }
  }
  return bad;
}

// The host FFT alone (sign +, unnormalised) of n values in place, for tests:
// x[m] = sum_l x[l] exp(+2 pi i l m / n).
int hostnufft_fft(double* re_im, int64_t n, int nthreads) {
  if (n < 1) return -1;
  BigFft b;
  make_bigfft(b, n);
  std::vector<cplx> x(n), s(1);
  for (int64_t i = 0; i < n; ++i) x[i] = cplx(re_im[2 * i], re_im[2 * i + 1]);
  bigfft(b, x.data(), s.data(), nthreads);
  for (int64_t m = 0; m < n; ++m) {
    const cplx& v = mode_at(b, x.data(), m);
    re_im[2 * m] = v.real();
    re_im[2 * m + 1] = v.imag();
  }
  return 0;
}

}  // extern "C"
