// Host simulation of the two-pass register-tile FFT (fft2_index.h): the
// threads of each workgroup run one after another, the LDS exchanges go
// through an array of the kernel's size (every slot access bounds-checked,
// every read slot must have been written in the same exchange), and the
// result is compared with the direct DFT X_m = sum_l x_l exp(+2 pi i l m / n)
// at sampled modes.  Usage: fft2_check L0 L1 C; prints "ok" on success.
#include <complex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2409_08090_amd/csrc/fft2_index.h"

using cd = std::complex<double>;
using namespace mils::fft2;

static cd root(long double x, long double N) {
  const long double a = 2.0L * 3.14159265358979323846264338327950288L * x / N;
  return cd((double)cosl(a), (double)sinl(a));
}

static void dft_r(cd* a, int R) {
  cd o[16];
  for (int k = 0; k < R; ++k) {
    cd acc = 0;
    for (int q = 0; q < R; ++q) acc += a[q] * root((long double)((q * k) % R), R);
    o[k] = acc;
  }
  for (int k = 0; k < R; ++k) a[k] = o[k];
}

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { std::printf(__VA_ARGS__); std::printf("\n"); ++fails; return; } } while (0)

// one line's stages on the registers of all its threads; lines share the LDS
// array `lds` at base line * pitch
static void run_line_stages(int L, int nthreads_line, std::vector<std::vector<cd>>& v,
                            std::vector<cd>& lds, std::vector<int>& stamp, int base, int& epoch) {
  const int TL = threads(L);
  if (nthreads_line != TL) { std::printf("thread count\n"); ++fails; return; }
  for (int s = 0; s < nstages(L); ++s) {
    const int R = radix(L, s), Ns = ns(L, s), NB = 16 / R;
    for (int t = 0; t < TL; ++t)
      for (int k = 0; k < NB; ++k) {
        const int b = t + TL * k;
        const int kb = b % Ns;
        for (int q = 1; q < R; ++q) v[t][reg(L, s, k, q)] *= root((long double)q * kb, (long double)Ns * R);
        dft_r(&v[t][reg(L, s, k, 0)], R);
      }
    if (s + 1 == nstages(L)) break;
    ++epoch;
    for (int t = 0; t < TL; ++t)
      for (int k = 0; k < NB; ++k)
        for (int q = 0; q < R; ++q) {
          const int p = out_pos(L, s, t + TL * k, q);
          const int slot = base + pad(p);
          CHECK(p >= 0 && p < L && slot >= base && slot < base + L + L / 16, "write slot L=%d s=%d p=%d", L, s, p);
          CHECK(stamp[slot] != epoch, "slot written twice L=%d s=%d p=%d", L, s, p);
          lds[slot] = v[t][reg(L, s, k, q)];
          stamp[slot] = epoch;
        }
    const int R2 = radix(L, s + 1), NB2 = 16 / R2;
    for (int t = 0; t < TL; ++t)
      for (int k = 0; k < NB2; ++k)
        for (int q = 0; q < R2; ++q) {
          const int p = in_pos(L, s + 1, t + TL * k, q);
          const int slot = base + pad(p);
          CHECK(p >= 0 && p < L && slot >= base && slot < base + L + L / 16, "read slot");
          CHECK(stamp[slot] == epoch, "read of an unwritten slot L=%d s=%d p=%d", L, s + 1, p);
          v[t][reg(L, s + 1, k, q)] = lds[slot];
        }
  }
}

// LDS bank pairs of the exchanges of C interleaved lines (lane l of a wave:
// column l mod C, thread l / C; C = 1: one line per wave): an 8-byte access
// of a wave is modelled as four cycles of 16 lanes over 16 bank pairs (32
// banks of 4 bytes), and a cycle whose lanes fall on the same pair at two
// different slots is a conflict.  Returns the number of conflicting cycles.
static int bank_conflicts(int L, int C, int pitch) {
  const int TL = threads(L), NT = C * TL;
  int bad = 0;
  for (int s = 0; s + 1 < nstages(L); ++s)
    for (int dir = 0; dir < 2; ++dir) {
      const int R = radix(L, dir ? s + 1 : s), NB = 16 / R;
      for (int k = 0; k < NB; ++k)
        for (int q = 0; q < R; ++q)
          for (int g0 = 0; g0 < NT; g0 += 16) {
            int slot_of_pair[16];
            for (int i = 0; i < 16; ++i) slot_of_pair[i] = -1;
            bool conflict = false;
            for (int tid = g0; tid < g0 + 16 && tid < NT; ++tid) {
              const int c = tid % C, t = tid / C;
              const int p = dir ? in_pos(L, s + 1, t + TL * k, q) : out_pos(L, s, t + TL * k, q);
              const int slot = c * pitch + pad(p);
              int& o = slot_of_pair[slot % 16];
              if (o >= 0 && o != slot) conflict = true;
              o = slot;
            }
            bad += conflict;
          }
    }
  return bad;
}

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  const int L0 = std::atoi(argv[1]), L1 = std::atoi(argv[2]), C = std::atoi(argv[3]);
  if (!line_ok(L0) || !line_ok(L1) || L1 % C) { std::printf("bad sizes\n"); return 2; }
  const int64_t n = (int64_t)L0 * L1;
  std::mt19937_64 rng(L0 * 7 + L1);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<cd> x(n), mid(n), X(n, cd(NAN, NAN));
  for (auto& e : x) e = cd(nd(rng), nd(rng));
  {
    const int b0 = bank_conflicts(L0, C, line_pitch_c(L0, C)), b1 = bank_conflicts(L1, 1, line_pitch(L1));
    if (b0 || b1) {
      std::printf("LDS bank conflicts: first pass %d, last pass %d cycles\n", b0, b1);
      return 1;
    }
  }
  // first pass: column blocks of C columns, results stored row-major [L0][L1]
  {
    const int TL = threads(L0);
    std::vector<cd> lds((size_t)C * line_pitch_c(L0, C));
    std::vector<int> stamp(lds.size(), 0);
    int epoch = 0;
    for (int sb = 0; sb < L1 / C; ++sb) {
      const int s0 = sb * C;
      for (int c = 0; c < C; ++c) {
        std::vector<std::vector<cd>> v(TL, std::vector<cd>(16));
        for (int t = 0; t < TL; ++t)
          for (int q = 0; q < 16; ++q) v[t][q] = x[(int64_t)(t + q * TL) * L1 + s0 + c];
        run_line_stages(L0, TL, v, lds, stamp, c * line_pitch_c(L0, C), epoch);
        if (fails) return 1;
        for (int t = 0; t < TL; ++t)
          for (int r = 0; r < 16; ++r) {
            const int m0 = t + TL * final_j(L0, r);
            const cd w = root((long double)(s0 + c) * m0, (long double)n);
            mid[(int64_t)m0 * L1 + s0 + c] = v[t][r] * w;
          }
      }
    }
  }
  // last pass: one row m0 at a time
  {
    const int TL = threads(L1);
    std::vector<cd> lds(line_pitch(L1));
    std::vector<int> stamp(lds.size(), 0);
    int epoch = 0;
    for (int m0 = 0; m0 < L0; ++m0) {
      std::vector<std::vector<cd>> v(TL, std::vector<cd>(16));
      for (int t = 0; t < TL; ++t)
        for (int q = 0; q < 16; ++q) {
          const int s = t + q * TL;
          v[t][q] = mid[(int64_t)m0 * L1 + s];
        }
      run_line_stages(L1, TL, v, lds, stamp, 0, epoch);
      if (fails) return 1;
      for (int t = 0; t < TL; ++t)
        for (int r = 0; r < 16; ++r) {
          const int m1 = t + TL * final_j(L1, r);
          X[m0 + (int64_t)L0 * m1] = v[t][r];
        }
    }
  }
  // direct DFT at sampled modes
  double maxerr = 0.0, scale = 0.0;
  std::uniform_int_distribution<int64_t> pick(0, n - 1);
  for (int i = 0; i < 64; ++i) {
    const int64_t fixed[4] = {0, 1, n - 1, n / 2};
    const int64_t m = i < 4 ? fixed[i] : pick(rng);
    cd ref = 0;
    for (int64_t l = 0; l < n; ++l) ref += x[l] * root((long double)((l * m) % n), (long double)n);
    maxerr = std::max(maxerr, std::abs(X[m] - ref));
    scale = std::max(scale, std::abs(ref));
  }
  for (int64_t m = 0; m < n; ++m)
    if (std::isnan(X[m].real())) { std::printf("mode %lld not written\n", (long long)m); return 1; }
  std::printf("L0=%d L1=%d C=%d max error %.3e (scale %.3e)\n", L0, L1, C, maxerr, scale);
  if (!(maxerr <= 1e-12 * scale)) return 1;
  std::printf("ok\n");
  return 0;
}
