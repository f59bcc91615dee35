// mils_internal.h -- plan and argument structures shared by the host runtime
// and the HIP kernels of libmils (gfx950).  Everything here is plain data
// passed to kernels by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mils {

constexpr int kMaxPass = 4;
constexpr int kMaxRadixStages = 12;

// One FFT pass of the multi-pass Stockham transform.  The grid of n cells is
// viewed as [P][L][S] (P = product of the earlier lengths, S of the later
// ones); the pass takes length-L transforms along the middle axis, multiplies
// output k of column s by exp(+2 pi i s k / (L S)) and stores element
// (p, k, s) at k*(P*S) + p*S + s, so that after the last pass row p holds
// the outputs m = p + P*k.
struct FftPass {
  int L;
  int C;                   // columns (S-direction) per workgroup; rows per workgroup in the last pass
  int cshift;              // log2(C) for the first/middle passes (C is a power of two)
  int64_t P, S;
  int nrad;
  int rad[kMaxRadixStages];
  int64_t twL_off;         // exp(2 pi i x / L), x in [0, L); two-level when big (see kTwLo)
  int big;                 // 1: a "big" pass (kThreadsBig threads, up to kLdsBig bytes of LDS)
  int64_t twlo_off;        // exp(2 pi i x / (L S)), x in [0, 2^bshift)
  int64_t twhi_off;        // exp(2 pi i (x << bshift) / (L S))
  int bshift;
};

// Plan of one NUFFT problem size (everything except the data).
struct Plan {
  int prec;                // 0 = FP64 grids, 1 = FP32 grids
  int64_t nf;              // number of output frequencies
  int64_t K;               // floor(nf / 2): output k <-> mode k - K
  int64_t n;               // fine grid size
  int w;                   // kernel width (cells)
  double beta;             // ES shape parameter
  double hw;               // w / 2
  double sigma;
  int npass;
  FftPass pass[kMaxPass];
  int64_t S1;              // row length of the spreading view [n / S1][S1]
  int64_t nrows;           // n / S1
  int T;                   // spreading tile (divides S1)
  int Tb;                  // bin width in cells (a power of two)
  int Tb_shift;            // log2(Tb)
  int64_t nbins;           // ceil(n / Tb)
  int D;                   // rows per workgroup of the last pass
  int fft2;                // 1: two-pass register-tile FFT (fft2.h), n = L0 * L1
  int64_t tw_count;        // complex entries in the twiddle buffer
  const void* hcoef;       // device: kernel polynomial coefficients (Real), see kHornerK
};

// The spreading kernel at the w cells of a point is evaluated as w
// polynomials in u = 2t - 1, t = the point's offset from its first cell
// (plan-owned table of kHornerN(prec) x kHornerK Reals, highest degree first,
// zero rows for k >= w).
constexpr int kHornerK = 20;                  // widest kernel (cells)
constexpr int kHornerN64 = 15, kHornerN32 = 9;  // coefficients per polynomial
__host__ __device__ constexpr inline int horner_n(int prec) { return prec == 1 ? kHornerN32 : kHornerN64; }

// Scalars produced on the device by the statistics kernel.
struct DevStats {
  double W;        // sum of weights
  double mu;       // weighted mean of y
  double M2;       // sum w (y - mu)^2
  double tmin, tmax;
  double tau;      // time origin subtracted before gridding
  double ysub;     // value subtracted from y (mu when centering, else 0)
  double Ybar;     // weighted mean of the data fed to the sums (0 when centred)
  double YY;       // normalising variance of the power
  int invalid;     // non-finite input or dy <= 0 seen
  int unsorted;    // t not non-decreasing
  int need_sort;   // points must go through the counting sort
  int status;      // 0 ok, -1 invalid input, -2 degenerate (YY == 0)
  int nill;        // frequencies whose fit is ill-posed (power NaN), counted by the last pass
  int nlow;        // frequencies evaluated directly near f = 0 (see lowfix)
  int64_t k_lo;    // first of them
};

// Per-call description of the data and output.
struct CallArgs {
  const double* t;
  const double* y;    // NULL for raw trig sums
  const double* dy;   // NULL = unit weights
  const double* h;    // raw trig sums strengths (NULL for periodograms)
  int64_t nd;
  int64_t nf;         // number of output frequencies
  double f0, df;
  double fch, fcl;    // f0 + K df as an unevaluated double-double
  int64_t kzero;      // output index with f == 0 exactly, or -1
  int norm;
  int center, fit_mean;
  // A fit whose determinant D = CC SS - CS^2 (sums normalised by the total
  // weight) is at most dmin is ill-posed at the transform's accuracy: its
  // power is NaN.  dmin = eps for transformed sums; sums evaluated directly
  // use only the relative test D <= 1e-12 CC SS.
  double dmin;
  int periodogram;    // 1: three grids + power; 0: one grid + complex sums
  int deterministic;  // fixed summation orders (bitwise-reproducible results)
  double* power;      // periodogram output
  double* sums;       // trig sums output (interleaved re/im)
  // Series sharing their weights (same t and dy): a weights-only call has
  // y == NULL (the statistics then take y = 0 and skip the constant-data
  // check) and unit_y set (the f-geometry strength is w^ e^{iwt}, the B
  // sum), and leaves B and B2 per output frequency in bsum_b, bsum_b2
  // (interleaved re/im, deconvolved).
  int unit_y;
  const double* bsum_b;
  const double* bsum_b2;
  // A series sharing its times with an earlier weights-only call: that
  // call's statistics (its sort decision holds for the series, and its bin
  // starts are still in the workspace unless the points must be sorted).
  const DevStats* wstats;
  // Last pass over nser (1..3) such series at once, grid g holding the A
  // sums of series g: its power, statistics and direct sums near f = 0.
  int nser;
  double* spow[3];
  const DevStats* sst[3];
  const double* slow[3];
};

// Device workspace of one call, carved from one allocation.
struct Work {
  DevStats* stats;
  double* partials;       // per-block partial reductions
  int* bin_start;         // nbins + 1
  int* bin_count;         // nbins + 1 (counting sort)
  int* bin_cursor;        // nbins
  int* scan_part;         // scan block sums
  double* ts;             // sorted copies (counting sort path)
  double* ys;
  double* dys;
  double* hs;
  unsigned char* rowflag_f;   // nrows
  unsigned char* rowflag_2f;  // nrows
  int* act_rows_f;            // nrows: active rows of geometry f, in order
  int* act_rows_2f;           // nrows: same for geometry 2f
  int* nact;                  // 2: number of active rows (f, 2f)
  void* grid[3];          // G grids of n complex
  void* grid2[3];         // second buffers for passes >= 2
  const void* tw;         // twiddles (plan-owned)
  const double* inv_phihat;  // 1 / phihat(|m|), m = 0..K (plan-owned)
  const double* inv_phihat2; // two-pass plans: 1 / phihat in last-pass order, n entries (plan-owned)
  void* f2out;               // two-pass plans: last-pass results, n doubles (power) or double2 (sums)
  double* lowpart;        // per-block partial direct sums near f = 0
  double* lowfix;         // direct sums A, B, B2 near f = 0: kLowParts rows of kLowMax x 6
  uint64_t* keys;         // det_keys(nd) sort keys of the reproducible binning
};

// Keys of the reproducible binning: the next power of two >= nd (>= 2).
inline int64_t det_keys(int64_t nd) {
  int64_t k = 2;
  while (k < nd) k <<= 1;
  return k;
}

constexpr int kStatsBlocks = 1024;
constexpr int kThreads = 256;       // threads of most kernels
// threads of the last FFT pass: FP64 blocks hold 4 rows of each grid, FP32
// blocks 8 (the radix-16 stages then keep most threads busy in both)
constexpr int kThreadsLast64 = 256, kThreadsLast32 = 512;
template <typename Real>
constexpr int last_threads() {
  return sizeof(Real) == 8 ? kThreadsLast64 : kThreadsLast32;
}
// Big passes: one workgroup of kThreadsBig threads per CU holds a column (or
// row) set of up to kEbig elements in LDS, so that two passes cover grids of
// ~1e7 cells.  Their in-pass twiddles come from a two-level table in LDS:
// exp(2 pi i x / L) = lo[x mod kTwLo] * hi[x / kTwLo].
constexpr int kThreadsBig = 1024;
constexpr int kEbig64 = 9600, kEbig32 = 19200;
constexpr size_t kLdsBig = 163840;  // LDS of one workgroup (gfx950)
constexpr int kTwLo = 64;
constexpr int kRowsMax = 16384;     // rows of the spreading view [nrows][S1]
__host__ __device__ constexpr inline int tw2_count(int L) { return kTwLo + (L + kTwLo - 1) / kTwLo; }
constexpr int kTileMax = 1024;      // spreading tile (cells)
constexpr int kSpreadGrid = 4096;   // workgroups of the persistent spread
constexpr int kLmax = 1024;         // longest per-pass FFT length
// elements held in LDS by one workgroup of a first/middle pass and of the last pass
constexpr int kEmid64 = 2048, kEmid32 = 4096;
constexpr int kElast64 = 3072, kElast32 = 6144;
// the persistent batched kernel runs every phase with 256 threads
// Near f = 0 (|f| * span < 2) the floating-mean terms CC = (1 + C2)/2 - C^2 etc.
// cancel and the 2x2 fit is ill-conditioned; there the three sums are
// evaluated directly (FP64, at most kLowMax frequencies) instead of read
// from the transform's band edge.
constexpr int kLowMax = 16;
constexpr int kLowGroup = 8;
constexpr int kLowBlocks = 512;
constexpr int kLowParts = 8;  // rows of lowfix (partial sums; the last pass adds them)

// LDS pitch of the last FFT pass: its rows are interleaved element by element
// with no padding.
__host__ __device__ constexpr inline int last_pitch(int rows) { return rows; }

}  // namespace mils
