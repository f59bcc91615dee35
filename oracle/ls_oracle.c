/*
 * ls_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, direct CPU evaluation of what the NUFFT Lomb-Scargle path
 * computes.  It exists so that tests and the CPU-baseline leg of the benchmark
 * can check the GPU library against an independent implementation.  Nothing in
 * the product library calls, links or includes this file, and this file uses
 * nothing from the product library.
 *
 * What it computes (nifty-ls paper, Sec. 1, Eq. 1 and Eq. 2):
 *   the weighted trigonometric sums  C_k + i S_k = sum_j h_j exp(+i 2 pi f_k t_j)
 *   on the cyclic frequency grid f_k = f0 + k*df, evaluated directly in
 *   O(N_d) work per frequency (the "direct evaluation" of Sec. 1 and the
 *   reference result of Sec. 2.2), and from those sums the Lomb-Scargle
 *   periodogram defined as the weighted least-squares fit of a sinusoid (plus
 *   an optional constant: the "floating mean") at every frequency.
 *
 * Precision choices (none of them is an approximation of the definition):
 *   - the phase f_k * t_j is formed in double-double arithmetic and reduced
 *     modulo one cycle exactly, so the argument passed to libm cos/sin is the
 *     exact phase of the given binary64 inputs to ~1e-16 of a cycle;
 *   - every sum over j is a Neumaier-compensated sum;
 *   - the small normal-equation system of the least-squares fit is solved by
 *     Cholesky factorisation in long double.
 * Build without -ffast-math and with -ffp-contract=off.
 *
 * Parity status of each entry point is documented beside it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- error-free transformations (Knuth two-sum, fma two-product) -------- */
static void two_sum(double a, double b, double *s, double *e) {
  double x = a + b;
  double bb = x - a;
  *e = (a - (x - bb)) + (b - bb);
  *s = x;
}

static void two_prod(double a, double b, double *p, double *e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}

/* ---- Neumaier compensated accumulator ---------------------------------- */
typedef struct {
  double s, c;
} nsum;

static void nadd(nsum *acc, double x) {
  double t = acc->s + x;
  if (fabs(acc->s) >= fabs(x))
    acc->c += (acc->s - t) + x;
  else
    acc->c += (x - t) + acc->s;
  acc->s = t;
}

static double nval(const nsum *acc) { return acc->s + acc->c; }

/* The frequency f_k = f0 + k*df as an unevaluated pair hi + lo (exact to
 * ~2^-106 relative).  Returns 1 for the zero frequency, read as the frequency
 * whose binary64 value fl(f0 + fl(k*df)) is zero (f0 == -fl(k*df)). */
static int freq_dd(double f0, double df, int64_t k, double *hi, double *lo) {
  double p, e1, s, e2;
  two_prod((double)k, df, &p, &e1);
  two_sum(f0, p, &s, &e2);
  *hi = s;
  *lo = e1 + e2;
  return (s == 0.0);
}

/* Phase of f*t in cycles, reduced to [-1/2, 1/2).  f is the pair (fh, fl). */
static double phase_cycles(double fh, double fl, double t) {
  double a, b;
  two_prod(fh, t, &a, &b);
  b += fl * t;
  double r = (a - floor(a)) + b; /* a - floor(a) is exact */
  r -= floor(r + 0.5);
  return r;
}

static const double TWO_PI = 6.283185307179586476925286766559;

/*
 * oracle_trig_sums: out_re[i] + i*out_im[i] = sum_j h[j] exp(+i 2 pi f t_j)
 * with f = f0 + kidx[i]*df.  (Eq. 1 with real weights h_j; Eq. 2 with the
 * sign of the exponent as printed.)
 * Pinned by: 50-digit brute force on tiny inputs, the Dirichlet-kernel closed
 * form for evenly spaced times, the N_d = 1 case and linearity in h.
 */
void oracle_trig_sums(const double *t, const double *h, int64_t nd, double f0,
                      double df, const int64_t *kidx, int64_t nk,
                      double *out_re, double *out_im) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nk; ++i) {
    double fh, fl;
    freq_dd(f0, df, kidx[i], &fh, &fl);
    nsum sc = {0, 0}, ss = {0, 0};
    for (int64_t j = 0; j < nd; ++j) {
      double r = phase_cycles(fh, fl, t[j]);
      double ang = TWO_PI * r;
      nadd(&sc, h[j] * cos(ang));
      nadd(&ss, h[j] * sin(ang));
    }
    out_re[i] = nval(&sc);
    out_im[i] = nval(&ss);
  }
}

/* Normalisations of the periodogram.  chi2_ref is the residual of the
 * reference model (the constant, or zero), chi2 the residual of the best fit
 * including the sinusoid at f. */
enum { NORM_STANDARD = 0, NORM_MODEL = 1, NORM_LOG = 2, NORM_PSD = 3 };

/* Cholesky solve of the SPD system M x = b (dimension m <= 3) in long double.
 * Returns b^T M^{-1} b, and sets *ok = 0 when a pivot is not positive or is
 * below rel_tol times its diagonal entry (an ill-posed fit). */
static long double quad_form_inv(long double M[3][3], const long double b[3],
                                 int m, long double rel_tol, int *ok) {
  long double L[3][3] = {{0}};
  *ok = 1;
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j <= i; ++j) {
      long double s = M[i][j];
      for (int q = 0; q < j; ++q) s -= L[i][q] * L[j][q];
      if (i == j) {
        if (!(s > rel_tol * M[i][i])) {
          *ok = 0;
          return 0.0L;
        }
        L[i][i] = sqrtl(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  }
  /* forward solve L z = b; then b^T M^{-1} b = |z|^2 */
  long double z[3];
  long double acc = 0.0L;
  for (int i = 0; i < m; ++i) {
    long double s = b[i];
    for (int q = 0; q < i; ++q) s -= L[i][q] * z[q];
    z[i] = s / L[i][i];
    acc += z[i] * z[i];
  }
  return acc;
}

/*
 * oracle_periodogram: the Lomb-Scargle periodogram at f = f0 + kidx[i]*df.
 *
 * Weights w_j = 1/dy_j^2 (w_j = 1 when dy is NULL).  With center_data the data
 * are replaced by y_j - ybar, ybar the weighted mean.  At each frequency the
 * model a cos(2 pi f t) + b sin(2 pi f t) [+ c when fit_mean] is fitted by
 * weighted least squares; chi2 is the minimum weighted residual and chi2_ref
 * the residual of the model without the sinusoid (the best constant when
 * fit_mean, else zero).  Power:
 *   standard  (chi2_ref - chi2) / chi2_ref
 *   model     (chi2_ref - chi2) / chi2
 *   log       ln(chi2_ref / chi2)
 *   psd       (chi2_ref - chi2) / 2
 * The sums it needs (sum_j w cos, w sin, w cos^2, w sin^2, w cos sin,
 * w y cos, w y sin) are each evaluated directly, term by term; none is derived
 * from another by a trigonometric identity.
 *
 * flag[i]: 0 = ok; 1 = f is exactly zero (power defined as 0);
 *          2 = the fit is ill-posed at this f (power set to NaN).
 * Returns 0, or -1 when chi2_ref is not positive (constant data).
 * Pinned by: 30-digit brute-force least squares on tiny inputs, power = 1 for
 * a noiseless sinusoid, the classical DFT periodogram for evenly spaced unit
 * weights at integer frequencies, and the symmetry / invariance properties of
 * the fit.
 */
int oracle_periodogram(const double *t, const double *y, const double *dy,
                       int64_t nd, double f0, double df, const int64_t *kidx,
                       int64_t nk, int normalization, int center_data,
                       int fit_mean, double *power, int32_t *flag) {
  double *w = (double *)malloc(sizeof(double) * (size_t)nd);
  double *yt = (double *)malloc(sizeof(double) * (size_t)nd);
  if (!w || !yt) {
    free(w);
    free(yt);
    return -2;
  }
  nsum sw = {0, 0}, swy = {0, 0};
  for (int64_t j = 0; j < nd; ++j) {
    w[j] = dy ? 1.0 / (dy[j] * dy[j]) : 1.0;
    nadd(&sw, w[j]);
    nadd(&swy, w[j] * y[j]);
  }
  double W = nval(&sw);
  double ybar = nval(&swy) / W;
  nsum s1 = {0, 0}, s2 = {0, 0};
  for (int64_t j = 0; j < nd; ++j) {
    yt[j] = center_data ? y[j] - ybar : y[j];
    nadd(&s1, w[j] * yt[j]);
    nadd(&s2, w[j] * yt[j] * yt[j]);
  }
  long double Wy = nval(&s1), Wyy = nval(&s2);
  long double chi2_ref = fit_mean ? Wyy - Wy * Wy / (long double)W : Wyy;
  if (!(chi2_ref > 0.0L)) {
    free(w);
    free(yt);
    return -1;
  }

#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nk; ++i) {
    double fh, fl;
    if (freq_dd(f0, df, kidx[i], &fh, &fl)) {
      power[i] = 0.0;
      flag[i] = 1;
      continue;
    }
    nsum c = {0, 0}, s = {0, 0}, cc = {0, 0}, ss = {0, 0}, cs = {0, 0},
         yc = {0, 0}, ys = {0, 0};
    for (int64_t j = 0; j < nd; ++j) {
      double r = phase_cycles(fh, fl, t[j]);
      double ang = TWO_PI * r;
      double cj = cos(ang), sj = sin(ang);
      nadd(&c, w[j] * cj);
      nadd(&s, w[j] * sj);
      nadd(&cc, w[j] * cj * cj);
      nadd(&ss, w[j] * sj * sj);
      nadd(&cs, w[j] * cj * sj);
      nadd(&yc, w[j] * yt[j] * cj);
      nadd(&ys, w[j] * yt[j] * sj);
    }
    /* normal equations of the basis (cos, sin[, 1]) */
    long double M[3][3], b[3];
    int m = fit_mean ? 3 : 2;
    M[0][0] = nval(&cc);
    M[0][1] = M[1][0] = nval(&cs);
    M[1][1] = nval(&ss);
    b[0] = nval(&yc);
    b[1] = nval(&ys);
    if (fit_mean) {
      M[0][2] = M[2][0] = nval(&c);
      M[1][2] = M[2][1] = nval(&s);
      M[2][2] = W;
      b[2] = Wy;
    }
    int ok;
    long double explained = quad_form_inv(M, b, m, 1e-12L, &ok);
    if (!ok) {
      power[i] = NAN;
      flag[i] = 2;
      continue;
    }
    long double delta = fit_mean ? explained - Wy * Wy / (long double)W
                                 : explained;
    long double chi2 = chi2_ref - delta;
    long double p;
    switch (normalization) {
    case NORM_MODEL:
      p = delta / chi2;
      break;
    case NORM_LOG:
      p = logl(chi2_ref / chi2);
      break;
    case NORM_PSD:
      p = 0.5L * delta;
      break;
    default:
      p = delta / chi2_ref;
      break;
    }
    power[i] = (double)p;
    flag[i] = 0;
  }
  free(w);
  free(yt);
  return 0;
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
