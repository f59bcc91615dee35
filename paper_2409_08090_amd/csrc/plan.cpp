// plan.cpp -- the planner of libmils.
//
// The paper (Sec. 1) sets the kernel width and fine-grid size from the user
// tolerance eps.  Here: for upsampling factor sigma, the exponential-of-
// semicircle kernel of width w has aliasing error ~ exp(-pi w sqrt(1 - 1/sigma))
// (the published heuristic of the finufft papers the method builds on), so
// w = ceil(ln(1/eps) / (pi sqrt(1 - 1/sigma))) and beta = 0.97 pi w (1 - 1/(2 sigma)).
// The grid size n >= sigma * nf is the cheapest 5-smooth number that factors
// into LDS-resident passes of the Stockham FFT.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>

namespace mils {

namespace {

constexpr int kTileMaxCells = kTileMax;  // spreading tile (LDS accumulator)
constexpr int kMaxWidth = 20;            // widest spreading kernel
constexpr int kLmaxPass = kLmax;         // longest per-pass FFT length
constexpr size_t kLdsMax = 65536;        // dynamic LDS of one workgroup

// LDS of the last pass for d rows of length L of G grids (interleaved rows at
// pitch last_pitch(G d), plus L twiddles) fits one workgroup.
static bool last_lds_ok(int G, int d, int L, int prec) {
  const size_t elem = prec == 1 ? 8 : 16;
  return elem * ((size_t)L * (size_t)last_pitch(G * d) + (size_t)L) <= kLdsMax;
}

// Big passes (see kThreadsBig).  Columns per workgroup of a big first pass
// (0 if none fits): the most contiguous columns (a power of two up to 8, at
// least cmin) whose L x C tile, twiddles and row flags fit the LDS.
static int big_cols(int L, int64_t S, int prec, int cmin) {
  const size_t elem = prec == 1 ? 8 : 16;
  const int emax = prec == 1 ? kEbig32 : kEbig64;
  for (int c = 8; c >= cmin; c /= 2) {
    if (c > S || (int64_t)L * c > emax) continue;
    if (elem * ((size_t)L * c + tw2_count(L)) + (size_t)L + 64 <= kLdsBig) return c;
  }
  return 0;
}
// Rows per workgroup of a big last pass over G grids (0 if none fits).
static int big_rows(int L, int64_t P, int G, int prec) {
  const size_t elem = prec == 1 ? 8 : 16;
  const int emax = prec == 1 ? kEbig32 : kEbig64;
  for (int d = 8; d >= 1; d /= 2) {
    if (d > P || (int64_t)G * d * L > emax) continue;
    if (elem * ((size_t)G * d * L + tw2_count(L)) <= kLdsBig) return d;
  }
  return 0;
}
// Big passes are opt-in (MILS_FFT_BIG=1, read whenever a plan is made):
// one workgroup per CU cannot overlap its loads, transform and stores, and
// measured slower than three small passes on the 1.5e7-cell grids.
static bool big_enabled() {
  const char* e = std::getenv("MILS_FFT_BIG");
  return e && e[0] == '1';
}

std::vector<int64_t> smooth_in_range(int64_t lo, int64_t hi) {
  std::vector<int64_t> v;
  for (int64_t a = 1; a <= hi; a *= 2)
    for (int64_t b = a; b <= hi; b *= 3)
      for (int64_t c = b; c <= hi; c *= 5)
        if (c >= lo) v.push_back(c);
  std::sort(v.begin(), v.end());
  return v;
}

bool is_smooth(int64_t x) {
  if (x < 1) return false;
  for (int f : {2, 3, 5})
    while (x % f == 0) x /= f;
  return x == 1;
}

// radix plan of a 5-smooth length: radix 16, 8 and 4 first, then 2, 5, 3.
int radix_plan(int L, int* rad) {
  int n = 0;
  while (L % 16 == 0) {
    rad[n++] = 16;
    L /= 16;
  }
  while (L % 8 == 0 && L > 8) {
    rad[n++] = 8;
    L /= 8;
  }
  while (L % 4 == 0) {
    rad[n++] = 4;
    L /= 4;
  }
  while (L % 8 == 0) {
    rad[n++] = 8;
    L /= 8;
  }
  while (L % 2 == 0) {
    rad[n++] = 2;
    L /= 2;
  }
  while (L % 5 == 0) {
    rad[n++] = 5;
    L /= 5;
  }
  while (L % 3 == 0) {
    rad[n++] = 3;
    L /= 3;
  }
  return n;
}

int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// Split m into k factors, each a 5-smooth length in [2, lmax]; prefers
// balanced factors (largest minimal columns per workgroup).  Returns false
// when impossible.
bool split_mid(int64_t m, int k, int lmax, std::vector<int>* out) {
  if (k == 0) return m == 1;
  if (k == 1) {
    if (m >= 2 && m <= lmax && is_smooth(m)) {
      out->push_back((int)m);
      return true;
    }
    return false;
  }
  if (m < ((int64_t)1 << k)) return false;
  {
    double cap = std::pow((double)lmax, (double)k);
    if ((double)m > cap * (1.0 + 1e-12)) return false;
  }
  // target ~ m^(1/k); try divisors closest to it first
  double target = std::pow((double)m, 1.0 / k);
  std::vector<int> cands;
  for (int L = 2; L <= lmax; ++L)
    if (m % L == 0 && is_smooth(L)) cands.push_back(L);
  std::sort(cands.begin(), cands.end(), [&](int a, int b) {
    return std::fabs(std::log(a / target)) < std::fabs(std::log(b / target));
  });
  for (int L : cands) {
    std::vector<int> rest;
    if (split_mid(m / L, k - 1, lmax, &rest)) {
      out->push_back(L);
      out->insert(out->end(), rest.begin(), rest.end());
      return true;
    }
  }
  return false;
}

}  // namespace

// sigma = 1.25 in both precisions (the grid size then rounds up to the next
// smooth size: 1.31 for the 1.2e7-frequency grids).  FP32 rounding of the
// grid is amplified by 1/phihat at the band edge, which grows as sigma
// falls; at 1.31 the FP32 periodograms measured stay 35x or more below the
// 1e-4 bound, and the grid is 15% smaller than at 1.5.
double default_sigma(int prec) {
  (void)prec;
  return 1.25;
}


// Safety factor between the requested tolerance and the kernel's error
// estimate.  The estimate exp(-pi w sqrt(1 - 1/sigma)) runs ~1.6x below the
// measured worst-case error of the sums, and in FP64 the lowest frequencies of
// a floating-mean periodogram (f span ~ 0.2, where the cos and sin columns are
// nearly collinear) sit at the band edge of the transform and amplify it
// further; FP32 accuracy is bounded by its rounding instead.
static double width_margin(int prec) { return prec == 1 ? 2.0 : 8.0; }

int kernel_width(double eps, double sigma, int prec) {
  double w = std::ceil(std::log(width_margin(prec) / eps) /
                       (M_PI * std::sqrt(1.0 - 1.0 / sigma)));
  int wi = (int)w;
  return std::min(kMaxWidth, std::max(2, wi));
}

// Upsampling factor for a tolerance: the precision's default -- except 1.5
// for batched FP32 series, whose many small grids gained less from the
// smaller grid than they lost to the wider kernel (10^4-series batch 21.7 ms
// at 1.5, 22.3-22.5 ms at 1.25) -- or 2 when that would need a kernel wider
// than kMaxWidth cells.
static double choose_sigma(double eps, int prec, bool batch) {
  const double s = (batch && prec == 1) ? 1.5 : default_sigma(prec);
  const double w = std::log(width_margin(prec) / eps) / (M_PI * std::sqrt(1.0 - 1.0 / s));
  return w > kMaxWidth ? 2.0 : s;
}

double planner_sigma(double eps, int prec, bool batch) { return choose_sigma(eps, prec, batch); }

double kernel_beta(int w, double sigma) { return 0.97 * M_PI * w * (1.0 - 1.0 / (2.0 * sigma)); }

bool make_plan(const PlanRequest& r, Plan* out, std::string* err) {
  Plan p{};
  p.prec = r.prec;
  p.nf = r.nf;
  p.K = r.nf / 2;
  const double smin = r.sigma > 1.0 ? r.sigma : choose_sigma(r.eps, r.prec, r.batch);
  const int wguess = kernel_width(r.eps, smin, r.prec);
  int64_t nmin = (int64_t)std::ceil(smin * (double)r.nf);
  nmin = std::max<int64_t>(nmin, 2 * wguess + 2);
  nmin = std::max<int64_t>(nmin, 16);
  const int G = r.G;
  const int emid = r.prec == 1 ? kEmid32 : kEmid64;
  const int elast = r.prec == 1 ? kElast32 : kElast64;
  const int dmin = 4;
  const int cmax = 32;

  std::vector<int64_t> cand = r.n_fixed > 0 ? std::vector<int64_t>{r.n_fixed}
                                             : smooth_in_range(nmin, 2 * nmin + 64);
  const int big_cmin = r.prec == 1 ? 4 : 2;
  // Factorisation of n into np passes that fit (lens; big: two big passes).
  auto factor = [&](int np, int64_t n, std::vector<int>* lens, bool* big) -> bool {
    lens->clear();
    *big = false;
    if (np == 1) {
      if (G * n <= elast && n <= kLmaxPass && last_lds_ok(G, 1, (int)n, r.prec)) {
        lens->push_back((int)n);
        return true;
      }
      return false;
    }
    // last length: largest with >= dmin rows per workgroup
    const int llast_max = std::min<int64_t>(elast / (G * dmin), kLmaxPass);
    for (int Ll = llast_max; Ll >= 2; --Ll) {
      if (n % Ll || !is_smooth(Ll) || !last_lds_ok(G, dmin, Ll, r.prec)) continue;
      std::vector<int> mids;
      if (split_mid(n / Ll, np - 1, std::min(kLmaxPass, emid / 4), &mids)) {
        *lens = mids;
        lens->push_back(Ll);
        return true;
      }
    }
    // two big passes n = L0 * L1: most contiguous first-pass columns, then
    // most rows per last-pass workgroup
    if (np == 2 && !r.batch && big_enabled()) {
      int bc = 0, bd = 0, bl = 0;
      const int64_t l0_lo = std::max<int64_t>(2, (n + kEbig32 - 1) / kEbig32);
      const int64_t l0_hi = std::min<int64_t>(kEbig32, n / 2);
      for (int64_t L0 = l0_lo; L0 <= l0_hi; ++L0) {
        if (n % L0 || !is_smooth(L0)) continue;
        const int64_t L1 = n / L0;
        if (L1 > kEbig32) continue;
        const int c = big_cols((int)L0, L1, r.prec, big_cmin);
        const int d = c ? big_rows((int)L1, L0, G, r.prec) : 0;
        if (!c || !d) continue;
        if (c > bc || (c == bc && d > bd)) {
          bc = c;
          bd = d;
          bl = (int)L0;
        }
      }
      if (bl) {
        *lens = {bl, (int)(n / bl)};
        *big = true;
        return true;
      }
    }
    return false;
  };
  // Estimated time of a plan, in units of one FFT pass over one cell
  // (calibrated on the 1.5e7-cell grids): a first pass weighs 0.8, a middle
  // pass 1.1, the last pass 1.0 and a single in-LDS pass 0.3, each 7% more
  // (less) per radix stage above (below) four and 15% per halving of the row
  // pieces below 128 B; the spread adds ~0.049 w per
  // frequency (points ~ N_f / 12, the usual sampling).  Among the smooth sizes
  // up to 1.3 x the minimum this trades a slightly larger grid for fewer
  // stages and a narrower kernel.
  auto estimate = [&](int64_t n, const std::vector<int>& lens) -> double {
    const int np = (int)lens.size();
    int rad[kMaxRadixStages];
    double sum = 0.0;
    const int elem = r.prec == 1 ? 8 : 16;
    for (int i = 0; i < np; ++i) {
      const double wt = np == 1 ? 0.3 : (i == 0 ? 0.8 : (i + 1 == np ? 1.0 : 1.1));
      const int st = radix_plan(lens[i], rad);
      double f = wt * (1.0 + 0.07 * (st - 4));
      // a first/middle pass moves rows of C columns: below 128 B per row
      // piece each halving costs ~15%
      if (np > 1 && i + 1 < np) {
        const int c = std::min(cmax, pow2_floor(emid / lens[i]));
        for (int bytes = c * elem; bytes < 128; bytes *= 2) f *= 1.15;
      }
      sum += f;
    }
    const int wn = kernel_width(r.eps, (double)n / (double)r.nf, r.prec);
    return (double)n * sum + 0.049 * wn * (double)r.nf;
  };
  double best_cost = 1e300;
  int best_np = 0;
  int64_t best_n = 0;
  bool best_big = false;
  std::vector<int> best_len;
  const double nlim = 1.3 * (double)nmin;
  for (int64_t n : cand) {
    if (best_np && (double)n > nlim) break;
    for (int np = 1; np <= kMaxPass; ++np) {
      std::vector<int> lens;
      bool big = false;
      if (!factor(np, n, &lens, &big)) continue;
      const double cost = estimate(n, lens);
      if (cost < best_cost) {
        best_cost = cost;
        best_np = np;
        best_n = n;
        best_big = big;
        best_len = lens;
      }
      break;  // more passes over the same n only cost more
    }
  }
  if (!best_np) {
    if (err) *err = "no supported FFT factorisation for this number of frequencies";
    return false;
  }
  // Two-pass register-tile FFT (fft2.h) in place of plans of three or more
  // passes: n = L0 L1 with register-tile lines (L0 in 2048..8192; L1 in
  // 2048..4096 for three grids, to 8192 for one), estimated at 0.55 (first
  // pass: pruned reads, contiguous writes) + 1.0 (last pass) + 0.15 (the
  // transpose of the results) of one pass over the grid.
  int f2_l0 = 0, f2_l1 = 0;
  if (r.fft2 && best_np >= 3 && (G == 1 || G == 3)) {
    double f2_cost = 1e300;
    int64_t f2_n = 0;
    for (int64_t n : cand) {
      if ((double)n > nlim) break;
      // L0 = 4096 first: its first pass takes 4 columns (64-byte pieces for
      // the last pass's reads); 8192 x 2048 measured slower at n = 2^24
      for (int L0 : {4096, 8192, 2048}) {
        if (n % L0) continue;
        const int64_t L1 = n / L0;
        if (!(L1 == 2048 || L1 == 4096 || (G == 1 && L1 == 8192))) continue;
        const int wn = kernel_width(r.eps, (double)n / (double)r.nf, r.prec);
        const double cost = (double)n * 1.7 + 0.049 * wn * (double)r.nf;
        if (cost < f2_cost) {
          f2_cost = cost;
          f2_n = n;
          f2_l0 = L0;
          f2_l1 = (int)L1;
        }
        break;
      }
    }
    if (f2_n) {
      best_n = f2_n;
      best_np = 2;
      best_big = false;
      best_len = {f2_l0, f2_l1};
    } else {
      f2_l0 = 0;
    }
  }
  p.n = best_n;
  p.sigma = (double)best_n / (double)r.nf;
  p.w = kernel_width(r.eps, p.sigma, r.prec);
  // a grid that fits one workgroup costs nothing extra with the widest kernel,
  // and tiny problems (a handful of frequencies, huge sigma) need the margin:
  // the floating-mean cancellation at the lowest frequencies amplifies the
  // error of the sums there
  if (best_np == 1) p.w = std::max(p.w, std::min<int>(kMaxWidth, (int)(best_n / 2) - 1));
  p.beta = kernel_beta(p.w, p.sigma);
  p.hw = 0.5 * p.w;
  p.npass = best_np;
  int64_t before = 1;
  p.fft2 = f2_l0 ? 1 : 0;
  for (int i = 0; i < best_np; ++i) {
    FftPass& ps = p.pass[i];
    ps.L = best_len[i];
    ps.P = before;
    ps.S = best_n / (before * ps.L);
    before *= ps.L;
    ps.nrad = radix_plan(ps.L, ps.rad);
    ps.big = best_big ? 1 : 0;
    if (p.fft2) {
      // first pass: C columns per workgroup of L0 / 16 threads each (the
      // kernel's choice, at most 1024 threads); last pass: one row
      ps.C = i == 0 ? std::min(8, 16384 / ps.L) : 1;

      ps.cshift = 0;
      while ((1 << ps.cshift) < ps.C) ++ps.cshift;
      if (i == 1) p.D = 1;
      continue;
    }
    if (best_big) {
      if (i == 0) {
        ps.C = big_cols(ps.L, ps.S, r.prec, big_cmin);
        ps.cshift = 0;
        while ((1 << ps.cshift) < ps.C) ++ps.cshift;
      } else {
        ps.C = big_rows(ps.L, ps.P, G, r.prec);
        p.D = ps.C;
      }
      continue;
    }
    if (i + 1 < best_np) {
      int c = std::min(cmax, pow2_floor(emid / ps.L));
      while (c > 1 && c / 2 >= ps.S) c /= 2;
      ps.C = c;
      ps.cshift = 0;
      while ((1 << ps.cshift) < c) ++ps.cshift;
    } else {
      int d = 1;
      while (d < 8 && G * (2 * d) * ps.L <= elast && 2 * d <= ps.P &&
             last_lds_ok(G, 2 * d, ps.L, r.prec))
        d *= 2;
      if (G * d * ps.L > elast || !last_lds_ok(G, d, ps.L, r.prec)) {
        if (err) *err = "last FFT pass does not fit one workgroup";
        return false;
      }
      ps.C = d;
      p.D = d;
    }
  }
  if (best_np == 1) {
    p.S1 = best_n;
    p.nrows = 1;
  } else {
    p.nrows = p.pass[0].L;
    p.S1 = best_n / p.nrows;
    if (p.nrows > kRowsMax) {
      if (err) *err = "first FFT pass longer than the spreading view allows";
      return false;
    }
  }
  int T = 1;
  const int tmax = r.tile_max > 0 ? std::min(r.tile_max, kTileMaxCells) : kTileMaxCells;
  if (r.batch && r.tile_max > 0 && p.nrows > 1 && 2 * p.S1 <= tmax) {
    // batched series with an explicit tile cap (the batch autotuner's
    // candidates): a tile of several whole rows (the last one may be
    // shorter), so that short rows do not make many nearly empty tiles when
    // there are many series; without a cap a lone series keeps more, smaller
    // tiles
    T = (int)((tmax / p.S1) * p.S1);
  } else {
    for (int d = (int)std::min<int64_t>(p.S1, tmax); d >= 1; --d)
      if (p.S1 % d == 0) {
        T = d;
        break;
      }
  }
  p.T = T;
  p.Tb = best_n >= 4096 ? 32 : 8;
  p.Tb_shift = best_n >= 4096 ? 5 : 3;
  p.nbins = (best_n + p.Tb - 1) / p.Tb;
  if (out) *out = p;
  return true;
}

void make_twiddles(Plan* p, std::vector<double>* tw) {
  tw->clear();
  auto push_root = [&](int64_t x, int64_t N) {
    long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)x / (long double)N;
    tw->push_back((double)cosl(ang));
    tw->push_back((double)sinl(ang));
  };
  for (int i = 0; i < p->npass; ++i) {
    FftPass& ps = p->pass[i];
    ps.twL_off = (int64_t)(tw->size() / 2);
    if (ps.big || p->fft2) {
      for (int x = 0; x < kTwLo; ++x) push_root(x, ps.L);
      for (int h = 0; h < (ps.L + kTwLo - 1) / kTwLo; ++h) push_root((int64_t)h * kTwLo, ps.L);
    } else {
      for (int x = 0; x < ps.L; ++x) push_root(x, ps.L);
    }
    if (i + 1 < p->npass) {
      const int64_t N = (int64_t)ps.L * ps.S;
      int b = 0;
      while (((int64_t)1 << (2 * b)) < N) ++b;
      ps.bshift = b;
      const int64_t B = (int64_t)1 << b;
      ps.twlo_off = (int64_t)(tw->size() / 2);
      for (int64_t x = 0; x < B; ++x) push_root(x, N);
      ps.twhi_off = (int64_t)(tw->size() / 2);
      const int64_t nh = (N + B - 1) / B;
      for (int64_t x = 0; x < nh; ++x) push_root(x * B % N, N);
    } else {
      ps.bshift = 0;
      ps.twlo_off = ps.twhi_off = 0;
    }
  }
  p->tw_count = (int64_t)(tw->size() / 2);
}

void phihat_nodes(const Plan& p, std::vector<double>* z, std::vector<double>* gphi) {
  int q = 2 * p.w + 16;
  if (q % 2) ++q;
  z->clear();
  gphi->clear();
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 1; i <= q / 2; ++i) {
    long double x = cosl(pi * (i - 0.25L) / (q + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = x;
      for (int k = 2; k <= q; ++k) {
        long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (x * p1 - p0) / (x * x - 1.0L);
      long double dx = p1 / dp;
      x -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    {
      long double p0 = 1.0L, p1 = x;
      for (int k = 2; k <= q; ++k) {
        long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (x * p1 - p0) / (x * x - 1.0L);
    }
    long double g = 2.0L / ((1.0L - x * x) * dp * dp);
    long double phi = expl((long double)p.beta * (sqrtl(1.0L - x * x) - 1.0L));
    z->push_back((double)x);
    gphi->push_back((double)(g * phi));
  }
}

size_t layout_work(const Plan& p, int64_t nd, int G, char* base, Work* w, bool per_series) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~(size_t)255;
    char* ptr = base ? base + off : nullptr;
    off += bytes;
    return ptr;
  };
  Work x{};
  x.stats = reinterpret_cast<DevStats*>(take(sizeof(DevStats)));
  if (!per_series) x.partials = reinterpret_cast<double*>(take(sizeof(double) * 8 * kStatsBlocks));
  x.bin_start = reinterpret_cast<int*>(take(sizeof(int) * (p.nbins + 1)));
  x.bin_count = reinterpret_cast<int*>(take(sizeof(int) * (p.nbins + 1)));
  x.bin_cursor = reinterpret_cast<int*>(take(sizeof(int) * (p.nbins + 1)));
  const int64_t nchunks = (p.nbins + 1 + 2047) / 2048;
  x.scan_part = reinterpret_cast<int*>(take(sizeof(int) * (nchunks + 1)));
  x.ts = reinterpret_cast<double*>(take(sizeof(double) * nd));
  if (G == 3) {
    x.ys = reinterpret_cast<double*>(take(sizeof(double) * nd));
    x.dys = reinterpret_cast<double*>(take(sizeof(double) * nd));
  } else {
    x.hs = reinterpret_cast<double*>(take(sizeof(double) * nd));
  }
  if (!per_series) x.lowpart = reinterpret_cast<double*>(take(sizeof(double) * 6 * kLowMax * kLowBlocks));
  if (!per_series) x.keys = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * det_keys(nd)));
  x.lowfix = reinterpret_cast<double*>(take(sizeof(double) * 6 * kLowMax * (per_series ? 1 : kLowParts)));
  x.rowflag_f = reinterpret_cast<unsigned char*>(take(p.nrows));
  x.rowflag_2f = reinterpret_cast<unsigned char*>(take(p.nrows));
  if (!per_series) {
    x.act_rows_f = reinterpret_cast<int*>(take(sizeof(int) * p.nrows));
    x.act_rows_2f = reinterpret_cast<int*>(take(sizeof(int) * p.nrows));
    x.nact = reinterpret_cast<int*>(take(sizeof(int) * 2));
  }
  const size_t cbytes = p.prec == 1 ? 8 : 16;
  for (int g = 0; g < G; ++g) x.grid[g] = take(cbytes * p.n);
  if (p.npass >= 3 || p.fft2)
    for (int g = 0; g < G; ++g) x.grid2[g] = take(cbytes * p.n);
  if (p.fft2) x.f2out = take((G == 3 ? sizeof(double) : 2 * sizeof(double)) * p.n);
  off = (off + 255) & ~(size_t)255;
  if (w) *w = x;
  return off;
}

void make_horner(const Plan& p, std::vector<double>* coef) {
  const int N = horner_n(p.prec);
  const long double pi = 3.14159265358979323846264338327950288L;
  const long double hw = 0.5L * (long double)p.w;
  const long double beta = (long double)p.beta;
  coef->assign((size_t)N * kHornerK, 0.0);
  std::vector<long double> fv(N), ch(N), mono(N), tm1(N), t0(N), t1(N);
  for (int k = 0; k < p.w && k < kHornerK; ++k) {
    // samples at the Chebyshev points u_i of [-1, 1] (t = (u + 1) / 2)
    for (int i = 0; i < N; ++i) {
      const long double u = cosl(pi * (2 * i + 1) / (2.0L * N));
      const long double z = ((long double)k + 0.5L * (u + 1.0L)) / hw - 1.0L;
      const long double a = 1.0L - z * z;
      fv[i] = a >= 0 ? expl(beta * (sqrtl(a) - 1.0L)) : 0.0L;
    }
    for (int m = 0; m < N; ++m) {
      long double acc = 0;
      for (int i = 0; i < N; ++i) acc += fv[i] * cosl(pi * m * (2 * i + 1) / (2.0L * N));
      ch[m] = (m == 0 ? 1.0L : 2.0L) * acc / N;
    }
    // sum_m ch[m] T_m(u) as a polynomial in u (T_1 = u, T_{m+1} = 2u T_m - T_{m-1})
    std::fill(mono.begin(), mono.end(), 0.0L);
    std::fill(tm1.begin(), tm1.end(), 0.0L);
    std::fill(t0.begin(), t0.end(), 0.0L);
    t0[0] = 1.0L;  // T_0
    for (int m = 0; m < N; ++m) {
      for (int j = 0; j < N; ++j) mono[j] += ch[m] * t0[j];
      // t1 = T_{m+1}: u T_0 for m = 0, else 2 u T_m - T_{m-1}
      const long double two = m == 0 ? 1.0L : 2.0L;
      for (int j = 0; j < N; ++j) t1[j] = -tm1[j] + (j > 0 ? two * t0[j - 1] : 0.0L);
      tm1 = t0;
      t0 = t1;
    }
    for (int j = 0; j < N; ++j) (*coef)[(size_t)(N - 1 - j) * kHornerK + k] = (double)mono[j];
  }
}

}  // namespace mils
