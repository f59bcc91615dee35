// Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
// planner (plan.cpp: grid choice, FFT factorisations, twiddle tables, kernel
// transform nodes, kernel polynomials) over a sweep of sizes, tolerances and
// precisions, single-series, batched and two-pass plans; and the plain host
// NUFFT (hostnufft.cpp) on small periodograms, a batch and its FFT.  Built by
// tests/test_sanitize_host.py with -fsanitize=address,undefined and
// -fno-sanitize-recover=all, so any finding ends the program with an error.
// Prints "ok" at the end.
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../paper_2409_08090_amd/csrc/plan.h"

extern "C" {
int hostnufft_periodogram(const double* t, const double* y, const double* dy, int64_t nd,
                          double f0, double df, int64_t nf, double eps, int norm, int center,
                          int fit_mean, int nthreads, double* power);
int hostnufft_batch(int64_t ncurves, const int64_t* nd_off, const double* t, const double* y,
                    const double* dy, const int64_t* nf_off, const double* f0, const double* df,
                    double eps, int norm, int center, int fit_mean, int nthreads, double* power,
                    int32_t* status);
int hostnufft_fft(double* re_im, int64_t n, int nthreads);
}

using namespace mils;

static int planner_sweep() {
  int plans = 0;
  std::vector<double> tw, z, g, hc;
  for (int prec : {0, 1}) {
    for (double eps : {1e-5, 1e-9, 1e-12}) {
      if (prec == 1 && eps < 1e-6) continue;
      for (int64_t nf = 1; nf <= (int64_t)1 << 25; nf = nf * 3 / 2 + 1) {
        for (int mode = 0; mode < 3; ++mode) {
          PlanRequest r{nf, eps, prec, 3};
          r.batch = mode == 1;
          r.fft2 = mode == 2;
          Plan p{};
          std::string err;
          if (!make_plan(r, &p, &err)) continue;
          make_twiddles(&p, &tw);
          if (p.n <= (int64_t)1 << 22) {  // the node and polynomial tables
            phihat_nodes(p, &z, &g);
            make_horner(p, &hc);
          }
          if (p.n < nf || tw.size() != (size_t)(2 * p.tw_count)) {
            std::printf("plan nf=%lld prec=%d mode=%d: n=%lld tw=%zu\n", (long long)nf, prec,
                        mode, (long long)p.n, tw.size());
            return -1;
          }
          ++plans;
        }
      }
    }
  }
  return plans;
}

static int host_nufft() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::normal_distribution<double> nd(0.0, 1.0);
  // single series of ragged sizes, sorted and not, with and without dy
  for (int n : {1, 3, 17, 200, 1500}) {
    for (int64_t nf : {(int64_t)1, (int64_t)7, (int64_t)12 * n + 5}) {
      std::vector<double> t(n), y(n), dy(n), p(nf);
      for (int i = 0; i < n; ++i) {
        t[i] = 100.0 * u(rng);
        y[i] = std::sin(2.0 * M_PI * 0.37 * t[i]) + 0.1 * nd(rng);
        dy[i] = 0.5 + u(rng);
      }
      for (int norm = 0; norm < 4; ++norm) {
        const int rc = hostnufft_periodogram(t.data(), y.data(), norm % 2 ? nullptr : dy.data(),
                                             n, 0.002, 0.002, nf, norm == 3 ? 1e-5 : 1e-9, norm,
                                             1, 1, 2, p.data());
        if (rc != 0 && rc != -2) {
          std::printf("periodogram n=%d nf=%lld norm=%d rc=%d\n", n, (long long)nf, norm, rc);
          return 1;
        }
      }
    }
  }
  // a batch of uneven series
  const int m = 24;
  std::vector<int64_t> ndo(m + 1, 0), nfo(m + 1, 0);
  for (int i = 0; i < m; ++i) {
    ndo[i + 1] = ndo[i] + 5 + (int64_t)(400 * u(rng));
    nfo[i + 1] = nfo[i] + 12 * (ndo[i + 1] - ndo[i]);
  }
  std::vector<double> t(ndo[m]), y(ndo[m]), dy(ndo[m]), f0(m), df(m), p(nfo[m]);
  for (int64_t j = 0; j < ndo[m]; ++j) {
    t[j] = 50.0 * u(rng);
    y[j] = nd(rng);
    dy[j] = 1.0;
  }
  for (int i = 0; i < m; ++i) f0[i] = df[i] = 0.004;
  std::vector<int32_t> st(m);
  hostnufft_batch(m, ndo.data(), t.data(), y.data(), dy.data(), nfo.data(), f0.data(), df.data(),
                  1e-9, 0, 1, 1, 2, p.data(), st.data());
  // the FFT alone on 5-smooth and other lengths
  for (int64_t n : {1, 2, 3, 5, 7, 64, 100, 243, 1000, 4096, 15625}) {
    std::vector<double> x(2 * n);
    for (auto& e : x) e = nd(rng);
    if (hostnufft_fft(x.data(), n, 2) != 0) return 1;
  }
  return 0;
}

int main() {
  const int plans = planner_sweep();
  if (plans <= 0) return 1;
  if (host_nufft() != 0) return 1;
  std::printf("%d plans ok\n", plans);
  return 0;
}
