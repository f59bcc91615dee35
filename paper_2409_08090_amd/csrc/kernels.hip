// kernels.hip -- the HIP kernels of the NUFFT Lomb-Scargle path (gfx950).
//
// Path of one periodogram (nifty-ls paper, Sec. 1):
//   k_stats      weights, weighted mean / variance, time range, input checks
//   k_bins_*     point binning by fine-grid cell (sorted fast path, or a
//                counting sort)
//   k_spread     exponential-of-semicircle spreading onto the upsampled grid
//                (geometry f: data and weight strengths; geometry 2f: weights)
//   k_fft_pass   one pass of the multi-pass Stockham FFT through HBM
//   k_fft_last   last FFT pass fused with deconvolution (the diagonal
//                rescaling), crop to the requested modes and power assembly
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <type_traits>

#include "device_math.h"
#include "fft2.h"
#include "fft_core.h"
#include "index_math.h"
#include "kernels.h"
#include "mils_internal.h"
#include "path_device.h"

namespace mils {

// ============================================================================
// Statistics: weighted mean/variance (merged Welford moments), time range,
// sortedness and validity.  k_stats leaves one partial per block; the one-block
// k_stats_final combines them in a fixed order and writes the scalars of the
// call.  (Two launches instead of a last-block-done counter: the device-scope
// fence such a counter needs is paid by every block.)
// ============================================================================
struct StatsPart {
  Moments m;
  double lo, hi;
  int bad, uns;
};

// Block-wide combine of one StatsPart per thread; thread 0 gets the total.
__device__ __forceinline__ StatsPart stats_block_combine(StatsPart x) {
  __shared__ double sW[kThreads], sMu[kThreads], sM2[kThreads], sLo[kThreads], sHi[kThreads];
  __shared__ int sBad[kThreads], sUns[kThreads];
  const int tid = threadIdx.x;
  sW[tid] = x.m.W;
  sMu[tid] = x.m.mu;
  sM2[tid] = x.m.M2;
  sLo[tid] = x.lo;
  sHi[tid] = x.hi;
  sBad[tid] = x.bad;
  sUns[tid] = x.uns;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      Moments y = {sW[tid], sMu[tid], sM2[tid]};
      moments_merge(y, sW[tid + s], sMu[tid + s], sM2[tid + s]);
      sW[tid] = y.W;
      sMu[tid] = y.mu;
      sM2[tid] = y.M2;
      sLo[tid] = fmin(sLo[tid], sLo[tid + s]);
      sHi[tid] = fmax(sHi[tid], sHi[tid + s]);
      sBad[tid] |= sBad[tid + s];
      sUns[tid] |= sUns[tid + s];
    }
    __syncthreads();
  }
  StatsPart r;
  r.m = {sW[0], sMu[0], sM2[0]};
  r.lo = sLo[0];
  r.hi = sHi[0];
  r.bad = sBad[0];
  r.uns = sUns[0];
  return r;
}

__global__ __launch_bounds__(kThreads) void k_stats(CallArgs a, Work w) {
  const int tid = threadIdx.x;
  StatsPart x = {{0.0, 0.0, 0.0}, INFINITY, -INFINITY, 0, 0};
  const double* yv = a.periodogram ? a.y : a.h;
  for (int64_t j = (int64_t)blockIdx.x * kThreads + tid; j < a.nd; j += (int64_t)gridDim.x * kThreads) {
    double t = a.t[j];
    double y = yv ? yv[j] : 0.0;
    double wj = 1.0;
    if (a.dy) {
      double d = a.dy[j];
      if (!(d > 0.0) || !isfinite(d)) x.bad = 1;
      wj = 1.0 / (d * d);
    }
    if (!isfinite(t) || !isfinite(y) || !isfinite(wj)) x.bad = 1;
    if (j > 0 && t < a.t[j - 1]) x.uns = 1;
    x.lo = fmin(x.lo, t);
    x.hi = fmax(x.hi, t);
    moments_merge(x.m, wj, y, 0.0);
  }
  const StatsPart r = stats_block_combine(x);
  if (tid == 0) {
    double* p = w.partials + 8 * blockIdx.x;
    p[0] = r.m.W;
    p[1] = r.m.mu;
    p[2] = r.m.M2;
    p[3] = r.lo;
    p[4] = r.hi;
    p[5] = (double)r.bad;
    p[6] = (double)r.uns;
  }
}

__global__ __launch_bounds__(kThreads) void k_stats_final(CallArgs a, Work w, int nparts) {
  const int tid = threadIdx.x;
  StatsPart x = {{0.0, 0.0, 0.0}, INFINITY, -INFINITY, 0, 0};
  for (int b = tid; b < nparts; b += kThreads) {
    const double* p = w.partials + 8 * b;
    moments_merge(x.m, p[0], p[1], p[2]);
    x.lo = fmin(x.lo, p[3]);
    x.hi = fmax(x.hi, p[4]);
    x.bad |= (p[5] != 0.0);
    x.uns |= (p[6] != 0.0);
  }
  const StatsPart r = stats_block_combine(x);
  if (tid == 0) {
    DevStats* st = w.stats;
    st->W = r.m.W;
    st->mu = r.m.mu;
    st->M2 = r.m.M2;
    st->tmin = r.lo;
    st->tmax = r.hi;
    st->invalid = r.bad;
    st->unsorted = r.uns;
    st->need_sort = a.wstats ? a.wstats->need_sort : r.uns;
    st->tau = a.periodogram ? r.lo : 0.0;
    const double W = r.m.W;
    st->ysub = a.center ? r.m.mu : 0.0;
    st->Ybar = a.center ? 0.0 : r.m.mu;
    double YY = r.m.M2 / W;
    if (!a.fit_mean && !a.center) YY += r.m.mu * r.m.mu;
    st->YY = YY;
    int status = 0;
    if (r.bad) status = -1;
    else if (a.periodogram && a.y && !(YY > 0.0)) status = -2;
    st->status = status;
    st->nill = 0;
    st->nlow = 0;
    st->k_lo = 0;
  }
}

// ============================================================================
// Binning.  bin_start[b] = index of the first point (in the order the spread
// reads them) whose cell lies in bin b or later; bin_start[nbins] = nd.
// ============================================================================
// Sorted fast path: when the bins of consecutive points are non-decreasing,
// bin_start[b] is the first point whose bin is >= b.  The bins up to the
// first point's all start at point 0 and those after the last point's at nd:
// the whole grid writes them (they can be most of the grid: the frequency
// step makes the grid's period several times the time span).  Every other
// point j starts the bins (bin(j-1), bin(j)], so it computes its own and its
// predecessor's bin and writes those entries: each bin is written by exactly
// one point, and a run longer than 8 bins (a gap in the data) by the whole
// wave.  A descent sets need_sort instead, and the counting sort below
// rebuilds everything.
__global__ __launch_bounds__(kThreads) void k_bins_sorted(CallArgs a, Plan p, Work w) {
  const DevStats* st = w.stats;
  if (st->status != 0) return;
  if (a.wstats && !st->need_sort) return;  // the weights-only call's bins hold
  const int nd = (int)a.nd;
  const int nb = (int)p.nbins;
  const int64_t gtid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  // The histogram of the counting sort is cleared by every block, before any
  // early exit: need_sort may be raised by another block of this launch.
  for (int64_t i = gtid; i <= nb; i += stride) w.bin_count[i] = 0;
  if (st->need_sort) return;
  const double tau = st->tau;
  const int b_first = point_bin(a.t[0], tau, a.df, p);
  const int b_last = point_bin(a.t[nd - 1], tau, a.df, p);
  for (int64_t b = gtid; b <= nb; b += stride) {
    if (b <= b_first) w.bin_start[b] = 0;
    else if (b > b_last) w.bin_start[b] = nd;
  }
  const int lane = threadIdx.x & 63;
  // wave-uniform loop over points 1 .. nd-1: every lane takes part in the
  // ballot and the shuffles
  for (int64_t j0 = 1 + (int64_t)blockIdx.x * kThreads + (threadIdx.x - lane); j0 < nd;
       j0 += stride) {
    const int64_t j = j0 + lane;
    int lo = 0, hi = -1;  // the bins [lo, hi] that start at point j
    if (j < nd) {
      const int bp = point_bin(a.t[j - 1], tau, a.df, p);
      const int bc = point_bin(a.t[j], tau, a.df, p);
      if (bc < bp) atomicOr(&w.stats->need_sort, 1);
      else {
        lo = bp + 1;
        hi = bc;
      }
    }
    const bool run = hi - lo >= 8;
    if (!run)
      for (int b = lo; b <= hi; ++b) w.bin_start[b] = (int)j;
    unsigned long long runs = __ballot(run);
    while (runs) {
      const int src = __ffsll(runs) - 1;
      runs &= runs - 1;
      const int l = __shfl(lo, src, 64), h = __shfl(hi, src, 64);
      const int v = (int)(j0 + src);
      for (int b = l + lane; b <= h; b += 64) w.bin_start[b] = v;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_sort_hist(CallArgs a, Plan p, Work w) {
  const DevStats* st = w.stats;
  if (st->status != 0 || !st->need_sort) return;
  const double tau = st->tau;
  for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < a.nd;
       j += (int64_t)gridDim.x * kThreads)
    atomicAdd(&w.bin_count[point_bin(a.t[j], tau, a.df, p)], 1);
}

// Exclusive scan of bin_count[0..nbins] into bin_start, in three launches:
// per-chunk scans, a one-block scan of the chunk totals, then the offsets.
__global__ __launch_bounds__(kThreads) void k_scan1(Plan p, Work w) {
  const DevStats* st = w.stats;
  if (st->status != 0 || !st->need_sort) return;
  __shared__ int s[kThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  const int64_t cnt = p.nbins + 1;
  int v[8];
  int sum = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    int64_t i = base + threadIdx.x * 8 + q;
    v[q] = i < cnt ? w.bin_count[i] : 0;
    sum += v[q];
  }
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    int x = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += x;
    __syncthreads();
  }
  int run = s[threadIdx.x] - sum;  // exclusive prefix of this thread
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    int64_t i = base + threadIdx.x * 8 + q;
    if (i < cnt) w.bin_start[i] = run;
    run += v[q];
  }
  if (threadIdx.x == kThreads - 1) w.scan_part[blockIdx.x] = s[kThreads - 1];
}

// Offsets of the per-chunk scans: block b adds the totals of chunks 0..b-1
// (a few hundred values) to its chunk.
__global__ __launch_bounds__(kThreads) void k_scan3(Plan p, Work w) {
  const DevStats* st = w.stats;
  if (st->status != 0 || !st->need_sort) return;
  __shared__ int red[kThreads];
  int part = 0;
  for (unsigned b = threadIdx.x; b < blockIdx.x; b += kThreads) part += w.scan_part[b];
  red[threadIdx.x] = part;
  __syncthreads();
  for (int sft = kThreads / 2; sft > 0; sft >>= 1) {
    if ((int)threadIdx.x < sft) red[threadIdx.x] += red[threadIdx.x + sft];
    __syncthreads();
  }
  const int add = red[0];
  const int64_t cnt = p.nbins + 1;
  for (int q = 0; q < 8; ++q) {
    int64_t i = (int64_t)blockIdx.x * kScanChunk + q * kThreads + threadIdx.x;
    if (i < cnt) {
      int v = w.bin_start[i] + add;
      w.bin_start[i] = v;
      if (i < p.nbins) w.bin_cursor[i] = v;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_sort_scatter(CallArgs a, Plan p, Work w) {
  const DevStats* st = w.stats;
  if (st->status != 0 || !st->need_sort) return;
  const double tau = st->tau;
  for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < a.nd;
       j += (int64_t)gridDim.x * kThreads) {
    double t = a.t[j];
    int pos = atomicAdd(&w.bin_cursor[point_bin(t, tau, a.df, p)], 1);
    if (pos < 0 || pos >= a.nd) continue;  // cannot happen with a consistent histogram
    w.ts[pos] = t;
    if (a.periodogram) {
      w.ys[pos] = a.y ? a.y[j] : 0.0;
      w.dys[pos] = a.dy ? a.dy[j] : 1.0;
    } else {
      w.hs[pos] = a.h[j];
    }
  }
}

// ============================================================================
// Reproducible binning (deterministic calls): the points in the order of the
// keys bin << 32 | index, sorted by a bitonic network (the keys are distinct,
// so the order is unique), gathered into the sorted copies; bin_start by a
// binary search per bin.  Replaces the counting sort, whose order within a
// bin follows atomic arrivals.
// ============================================================================
__global__ __launch_bounds__(kThreads) void k_det_keys(CallArgs a, Plan p, Work w, int64_t nk) {
  const DevStats* st = w.stats;
  if (st->status != 0) return;
  const double tau = st->tau;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nk;
       i += (int64_t)gridDim.x * kThreads) {
    uint64_t key = ~(uint64_t)0;
    if (i < a.nd) key = ((uint64_t)(uint32_t)point_bin(a.t[i], tau, a.df, p) << 32) | (uint64_t)i;
    w.keys[i] = key;
  }
}

// One compare-exchange step (block size k, distance jj) of the ascending
// bitonic sort of nk keys (nk a power of two): each pair (i, i ^ jj) is taken
// by the thread of its lower index.
__global__ __launch_bounds__(kThreads) void k_det_bitonic(Work w, int64_t nk, int64_t k, int64_t jj) {
  if (w.stats->status != 0) return;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nk;
       i += (int64_t)gridDim.x * kThreads) {
    const int64_t l = i ^ jj;
    if (l <= i) continue;
    const uint64_t x = w.keys[i], y = w.keys[l];
    const bool up = (i & k) == 0;
    if ((x > y) == up) {
      w.keys[i] = y;
      w.keys[l] = x;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_det_gather(CallArgs a, Plan p, Work w) {
  DevStats* st = w.stats;
  if (st->status != 0) return;
  const int nd = (int)a.nd;
  const int nb = (int)p.nbins;
  const int64_t total = nd > nb + 1 ? nd : nb + 1;
  for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kThreads) {
    if (q < nd) {
      const int j = (int)(w.keys[q] & 0xffffffffu);
      w.ts[q] = a.t[j];
      if (a.periodogram) {
        w.ys[q] = a.y ? a.y[j] : 0.0;
        w.dys[q] = a.dy ? a.dy[j] : 1.0;
      } else {
        w.hs[q] = a.h[j];
      }
    }
    if (q <= nb) {
      // first position whose bin is >= q (nd if none)
      w.bin_start[q] =
          lower_bound_idx(nd, (int)q, [&](int j) { return (int)(w.keys[j] >> 32); });
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->need_sort = 1;  // the spread reads the copies
}

// ============================================================================
// Spreading.  A tile is T consecutive cells of one row of the [nrows][S1]
// view of the grid; its workgroup gathers every point whose kernel support
// (w cells around u) meets the tile, accumulates the kernel-weighted
// strengths in LDS and writes the tile once: no global atomics, no halo
// exchange, and the result does not depend on how tiles are scheduled.
// Rows that no kernel support reaches are not written (nor visited); their
// flag tells the first FFT pass to treat them as zero.
// ============================================================================
// Row classification for the spread: the flag of every row of a geometry
// (1 if a kernel support reaches it) and the list of active rows in order.
// The compaction is one workgroup of kRowThreads threads; thread i takes the
// rows [i*rpt, (i+1)*rpt) (rpt = ceil(nrows / kRowThreads)), so their order
// survives one scan of the per-thread counts.
constexpr int kRowThreads = 1024;
static_assert(kRowsMax <= kRowThreads * 32, "row flags of a thread fit one word");
// Row classes, in two launches for geometries geo0 .. geo0 + gridDim.y - 1
// (0: f, 1: 2f).  k_row_flags: one thread per row of the [nrows][S1] view
// sets its flag (whether any kernel support of the geometry reaches it);
// k_row_compact: one workgroup per geometry lists the active rows in order
// and stores their count in nact[geometry].
__global__ __launch_bounds__(256) void k_row_flags(Plan p, Work w, int nd, int geo0) {
  const DevStats* st = w.stats;
  if (st->status != 0) return;
  const int geo = geo0 + (int)blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= p.nrows) return;
  const int h = (int)ceil(p.hw) + 1;
  const bool active = geo == 0 ? row_active<1>(r, h, p, w.bin_start, nd)
                               : row_active<2>(r, h, p, w.bin_start, nd);
  (geo == 0 ? w.rowflag_f : w.rowflag_2f)[r] = (unsigned char)active;
}

__global__ __launch_bounds__(kRowThreads) void k_row_compact(Plan p, Work w, int geo0) {
  __shared__ int scan[kRowThreads];
  const DevStats* st = w.stats;
  if (st->status != 0) return;
  const int geo = geo0 + (int)blockIdx.x;
  const unsigned char* rowflag = geo == 0 ? w.rowflag_f : w.rowflag_2f;
  int* act_rows = geo == 0 ? w.act_rows_f : w.act_rows_2f;
  const int tid = threadIdx.x;
  const int nrows = (int)p.nrows;
  const int rpt = (nrows + kRowThreads - 1) / kRowThreads;
  const int r0 = tid * rpt;
  unsigned flags = 0;  // bit i: row r0 + i is active (rpt <= 32)
  int cnt = 0;
  for (int i = 0; i < rpt && r0 + i < nrows; ++i) {
    const int active = rowflag[r0 + i] != 0;
    flags |= (unsigned)active << i;
    cnt += active;
  }
  scan[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < kRowThreads; off <<= 1) {
    const int x = tid >= off ? scan[tid - off] : 0;
    __syncthreads();
    scan[tid] += x;
    __syncthreads();
  }
  int pos = scan[tid] - cnt;
  for (int i = 0; i < rpt && r0 + i < nrows; ++i)
    if ((flags >> i) & 1u) act_rows[pos++] = r0 + i;
  if (tid == kRowThreads - 1) w.nact[geo] = scan[tid];
}

static void enqueue_row_class(const Plan& p, const Work& w, int nd, int geo0, int ngeo,
                              hipStream_t s) {
  const unsigned nb = (unsigned)((p.nrows + 255) / 256);
  hipLaunchKernelGGL(k_row_flags, dim3(nb, (unsigned)ngeo), dim3(256), 0, s, p, w, nd, geo0);
  hipLaunchKernelGGL(k_row_compact, dim3((unsigned)ngeo), dim3(kRowThreads), 0, s, p, w, geo0);
}

// Spreading over the tiles of the active rows only (their list and count come
// from k_row_compact): a fixed grid of workgroups takes tiles blk, blk + grid,
// ...; every tile is written by exactly one workgroup, so the result does not
// depend on scheduling.  T divides the row length S1 here.
template <typename Real, int GEO, int NG, bool DET = false>
__global__ __launch_bounds__(kThreads) void k_spread_rows(CallArgs a, Plan p, Work w, int gbase,
                                                          const int* act_rows, int slot) {
  __shared__ double acc[NG * 2 * kTileMax];
  __shared__ int rb[8], re[8], sv[2];
  __shared__ SpreadRecords<Real, NG, kThreads> rec;
  const DevStats* stp = w.stats;
  if (stp->status != 0) return;
  const int tpr = (int)(p.S1 / p.T);
  const int ntile = w.nact[slot] * tpr;
  for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
    const int q = t / tpr;
    const int tile = act_rows[q] * tpr + (t - q * tpr);
    spread_tile<Real, GEO, NG, kThreads, true, DET>(tile, p.T, kTileMax, a, p, w, *stp, gbase,
                                                    nullptr, acc, rb, re, sv, rec);
  }
}

// ============================================================================
// FFT passes.
// ============================================================================
template <typename Real, int EMAX, int NT, bool TW2>
__global__ __launch_bounds__(NT) void k_fft_pass(PassBufs<Real> b, FftPass ps,
                                                 const typename cplx<Real>::T* tw,
                                                 const DevStats* st) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (st->status != 0) return;
  const int64_t blk = xcd_remap(blockIdx.x, (int64_t)gridDim.x);
  const int g = blockIdx.y;
  fft_pass_block<Real, EMAX, NT, TW2>(blk, b.in[g], b.out[g], b.rowflag[g], ps, tw, smem);
}

template <typename Real, int G, int EMAX, int NT, bool TW2>
__global__ __launch_bounds__(NT) void k_fft_last(PassBufs<Real> b, FftPass ps, Plan pl,
                                                 CallArgs a, const typename cplx<Real>::T* tw,
                                                 const double* inv_phihat, const DevStats* stp,
                                                 const double* lowfix) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (stp->status != 0) return;
  const int64_t nblk = (ps.P + ps.C - 1) / ps.C;
  const int64_t blk = xcd_remap(blockIdx.x, nblk);
  const DevStats st = *stp;
  fft_last_block<Real, G, EMAX, NT, TW2>(blk, b, ps, pl.n, pl.nf, pl.K, a, tw, inv_phihat, st,
                                         smem, G == 3 ? lowfix : nullptr, kLowParts,
                                         const_cast<int*>(&stp->nill));
}

// The last pass for a group of series sharing their weights (a.nser grids of
// A sums).  Workgroups of 512 threads are held to 128 registers, so that two
// of them share a CU.
template <typename Real, int G, int EMAX, int NT, bool TW2>
__global__ __launch_bounds__(NT, NT >= 512 ? 4 : 1) void k_fft_last_ser(
    PassBufs<Real> b, FftPass ps, Plan pl, CallArgs a, const typename cplx<Real>::T* tw,
    const double* inv_phihat, const DevStats* stp, const double* lowfix) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (stp->status != 0) return;
  const int64_t nblk = (ps.P + ps.C - 1) / ps.C;
  const int64_t blk = xcd_remap(blockIdx.x, nblk);
  const DevStats st = *stp;
  fft_last_block<Real, G, EMAX, NT, TW2, true>(blk, b, ps, pl.n, pl.nf, pl.K, a, tw, inv_phihat,
                                               st, smem, nullptr, kLowParts);
}

// Direct FP64 sums A, B, B2 at the (at most kLowMax) frequencies nearest
// f = 0 with |f| span < 2, all of them in one sweep over the points.  Blocks
// stride over the points and leave their totals in lowpart; the one-block
// k_lowfreq_final adds them up into lowfix.  Block totals are formed by a
// transpose through LDS, kLowChunk values at a time: every value is then
// summed by 8 threads over 32 entries each, and the 8 parts are combined
// across lanes (a fixed order, so the result does not depend on timing).
constexpr int kLowChunk = 32;
constexpr int kLowStride = kThreads + 8;  // row pitch: spreads the 8 parts over the banks
constexpr int kLowNV = 6 * kLowMax;
__global__ __launch_bounds__(kThreads) void k_lowfreq(CallArgs a, Work w) {
  static_assert(kLowNV % kLowChunk == 0 && kLowChunk * 8 == kThreads, "transpose shape");
  __shared__ double red[kLowChunk * kLowStride];
  const DevStats st = *w.stats;
  if (st.status != 0 || !a.periodogram) return;
  int64_t k_lo;
  int nlow;
  low_band(st, a.f0, a.df, a.nf, k_lo, nlow);
  if (nlow == 0) return;
  const int tid = threadIdx.x;
  double acc[kLowNV];
  low_accumulate<kLowMax>(a, st, k_lo, nlow, (int64_t)blockIdx.x * kThreads + tid,
                          (int64_t)gridDim.x * kThreads, acc);
  const int v = tid >> 3, part = tid & 7;
#pragma unroll
  for (int c = 0; c < kLowNV; c += kLowChunk) {
#pragma unroll
    for (int i = 0; i < kLowChunk; ++i) red[i * kLowStride + tid] = acc[c + i];
    __syncthreads();
    double sum = 0.0;
#pragma unroll 8
    for (int i = 0; i < kThreads / 8; ++i) sum += red[v * kLowStride + part + 8 * i];
    sum += __shfl_xor(sum, 1, 64);
    sum += __shfl_xor(sum, 2, 64);
    sum += __shfl_xor(sum, 4, 64);
    if (part == 0) w.lowpart[(size_t)blockIdx.x * kLowNV + c + v] = sum;
    __syncthreads();
  }
}

// Block r of kLowParts adds the block totals [r*nparts/kLowParts,
// (r+1)*nparts/kLowParts) into row r of lowfix (one workgroup alone could
// not read the partials faster than one CU's bandwidth); the last pass adds
// the rows.  Thread (x, pr) of 8 x kLowNV adds value x over the blocks of its
// share congruent to pr mod 8 with eight independent partial sums, then the 8
// parts of x are combined across lanes.  Fixed order throughout, so the
// result does not depend on timing.
constexpr int kLowFinalThreads = 8 * kLowNV;
__global__ __launch_bounds__(kLowFinalThreads) void k_lowfreq_final(CallArgs a, Work w,
                                                                    int nparts) {
  DevStats* stp = w.stats;
  const DevStats st = *stp;
  if (st.status != 0 || !a.periodogram) return;
  int64_t k_lo;
  int nlow;
  low_band(st, a.f0, a.df, a.nf, k_lo, nlow);
  if (nlow == 0) return;
  const int tid = threadIdx.x;
  const int x = tid >> 3, pr = tid & 7;
  const int r = blockIdx.x;
  const int b0 = (int)(((int64_t)nparts * r) / kLowParts);
  const int b1 = (int)(((int64_t)nparts * (r + 1)) / kLowParts);
  double part[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) part[u] = 0.0;
  int b = b0 + pr;
  for (; b + 56 < b1; b += 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) part[u] += w.lowpart[(size_t)(b + 8 * u) * kLowNV + x];
  }
  for (int u = 0; b < b1; b += 8, ++u) part[u & 7] += w.lowpart[(size_t)b * kLowNV + x];
  double sum = ((part[0] + part[1]) + (part[2] + part[3])) + ((part[4] + part[5]) + (part[6] + part[7]));
  sum += __shfl_xor(sum, 1, 64);
  sum += __shfl_xor(sum, 2, 64);
  sum += __shfl_xor(sum, 4, 64);
  if (pr == 0 && x < 6 * nlow) w.lowfix[r * kLowNV + x] = sum;
  if (r == 0 && tid == 0) {
    stp->k_lo = k_lo;
    stp->nlow = nlow;
  }
}

// 1 / phihat(m), m = 0..K, where phihat is the Fourier transform of the
// spreading kernel on the fine grid (cell units):
//   phihat(m) = (w/2) int_{-1}^{1} phi(z) cos(pi w z m / n) dz,
// by Gauss-Legendre quadrature (nodes z_r > 0 with weights g_r phi(z_r)).
__global__ __launch_bounds__(kThreads) void k_phihat(double* inv_phihat, int64_t K, double w,
                                                     double n, const double* z,
                                                     const double* gphi, int q) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i > K) return;
  const double alpha = (double)i * (M_PI * w / n);
  double s = 0.0;
  for (int r = 0; r < q; ++r) s += gphi[r] * cos(alpha * z[r]);
  inv_phihat[i] = 1.0 / (w * s);
}

// 1 / phihat in the order of the two-pass last pass: entry m0 L1 + m1 is the
// factor of mode m = m0 + L0 m1 (0 where m is cropped).
__global__ __launch_bounds__(kThreads) void k_phihat2(double* iphi2, const double* inv_phihat,
                                                      int L0, int L1, int64_t n, int64_t nf,
                                                      int64_t K) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t m0 = i / L1, m1 = i - m0 * L1;
  const int64_t k = fft2::crop(m0 + (int64_t)L0 * m1, n, nf, K);
  double v = 0.0;
  if (k >= 0) {
    const int64_t mm = k - K;
    v = inv_phihat[mm < 0 ? -mm : mm];
  }
  iphi2[i] = v;
}

// ============================================================================
// Two-pass register-tile FFT (fft2.h).
// ============================================================================
// First pass: the C columns s0 .. s0+C-1 of grid blockIdx.y; the rows whose
// flag is clear are zero and are not read.  Output: row-major [L0][L1],
// element (s, m0) at m0 L1 + s, multiplied by exp(2 pi i s m0 / n): the
// workgroup writes a C-element piece of every row (neighbouring column
// blocks run on one XCD, whose L2 joins their pieces), so that the last pass
// reads whole rows contiguously.
template <typename Real, int L0, int C, bool HALVES>
__global__ __launch_bounds__(C * L0 / 16, 4) void k_fft2_first(Fft2Bufs<Real> b, FftPass ps,
                                                             const typename cplx<Real>::T* tw,
                                                             const DevStats* st) {
  using T2 = typename cplx<Real>::T;
  using Lds = typename std::conditional<HALVES, Real, T2>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  if (st->status != 0) return;
  constexpr int TL = L0 / 16, NT = C * TL, LP = fft2::line_pitch_c(L0, C);
  static_assert(NT <= 1024 && (C & (C - 1)) == 0, "first-pass workgroup shape");
  const int tid = threadIdx.x;
  const int c = tid & (C - 1), t = tid / C;
  const int g = blockIdx.y;
  const int64_t sb = xcd_remap(blockIdx.x, (int64_t)gridDim.x);
  const int64_t L1 = ps.S;
  const int64_t s = sb * C + c;
  Lds* ex = reinterpret_cast<Lds*>(smem);
  T2* twl = reinterpret_cast<T2*>(smem + (size_t)C * LP * sizeof(Lds));
  // the flags of this thread's 16 rows straight from memory (every workgroup
  // of the grid reads the same L0 bytes, so they come from the cache), then
  // the rows' loads, and only then the twiddle table into LDS: staging the
  // flags in LDS put a barrier before every workgroup's first load (first
  // pass 317 -> 305 us FP64, 202 -> 187 us FP32 at 4096 x 4096)
  const unsigned char* rfg = b.rowflag[g];
  unsigned char fl[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) fl[q] = rfg[t + q * TL];
  T2 v[16];
  const T2* in = b.grid[g] + s;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int row = t + q * TL;
    v[q] = czero<T2>();
    if (fl[q]) v[q] = in[(int64_t)row * L1];
  }
  for (int x = tid; x < tw2_count(L0); x += NT) twl[x] = tw[ps.twL_off + x];
  __syncthreads();
  // inter-pass twiddles exp(2 pi i s m0 / n) of this thread's outputs
  // m0 = t + TL j: the first and the step from the two-level table, fetched
  // before the transform so that their latency overlaps it
  const int64_t mask = ((int64_t)1 << ps.bshift) - 1;
  const T2* tlo = tw + ps.twlo_off;
  const T2* thi = tw + ps.twhi_off;
  const int64_t q0 = s * t, qs = s * TL;
  const T2 w0 = cmul(thi[q0 >> ps.bshift], tlo[q0 & mask]);
  const T2 ws = cmul(thi[qs >> ps.bshift], tlo[qs & mask]);
  f2_line<L0, HALVES>(v, t, ex + c * LP, twl);
  T2* out = b.mid[g] + s;
  T2 tk = w0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    out[(int64_t)(t + TL * j) * L1] = cmul(v[f2_reg_of<L0>(j)], tk);
    tk = cmul(tk, ws);
  }
}

// Last pass: row m0 of each of the G grids (threads g * TL + t), read
// contiguously with streaming loads (each element is read once; marked so,
// the pass took 287 us instead of 331 at 4096 x 4096 in FP64).  G = 3: the grid-0 threads take
// B and B2 of their outputs from the other grids' threads (through LDS) and
// write the power of mode m = m0 + L0 m1 to out[m0 L1 + m1]; G = 1: the
// deconvolved sums (double2).  Cropped modes are not written.
template <typename Real, int L1, int G, int C, bool HALVES>
__global__ __launch_bounds__(G * L1 / 16, G == 3 ? 3 : 2) void k_fft2_last(Fft2Bufs<Real> b, FftPass ps, Plan pl,
                                                            CallArgs a,
                                                            const typename cplx<Real>::T* tw,
                                                            const double* iphi2,
                                                            const DevStats* stp,
                                                            const double* lowfix, void* outv) {
  using T2 = typename cplx<Real>::T;
  using Lds = typename std::conditional<HALVES, Real, T2>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  if (stp->status != 0) return;
  constexpr int TL = L1 / 16, NT = G * TL, LP = fft2::line_pitch(L1);
  static_assert(NT <= 1024, "last-pass workgroup shape");
  const int tid = threadIdx.x;
  const int g = tid / TL, t = tid - g * TL;
  const int64_t L0 = ps.P;
  const int64_t m0 = xcd_remap(blockIdx.x, (int64_t)gridDim.x);
  // power (G = 3): the grids' results gathered in LDS, all of them (FP32) or
  // half the outputs at a time (FP64), and the power of each output computed
  // by one of all the workgroup's threads
  constexpr int NR = (G == 3 && HALVES) ? 2 : 1;  // rounds over the outputs
  constexpr int MR = L1 / NR;                      // outputs per round
  constexpr int PPT = (MR + NT - 1) / NT;          // outputs per thread and round
  const size_t exb = (size_t)G * LP * sizeof(Lds);
  const size_t cbb = G == 3 ? (size_t)G * MR * sizeof(T2) : 0;
  Lds* ex = reinterpret_cast<Lds*>(smem);
  T2* twl = reinterpret_cast<T2*>(smem + (exb > cbb ? exb : cbb));
  T2 v[16];
  const T2* in = b.mid[g] + m0 * L1;
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = ld_stream(&in[t + q * TL]);
  // the kernel-transform factors of the outputs this thread finishes
  constexpr int NIP = G == 3 ? NR * PPT : 16;
  double ipv[NIP];
  {
    const double* ip = iphi2 + m0 * L1;
#pragma unroll
    for (int i = 0; i < NIP; ++i) {
      int m1;
      if constexpr (G == 3) m1 = (i / PPT) * MR + tid + NT * (i % PPT);
      else m1 = t + TL * i;
      // (factors of cropped modes are not read)
      ipv[i] = (G != 3 || (tid + NT * (i % PPT)) < MR) &&
                       fft2::crop(m0 + L0 * m1, pl.n, a.nf, pl.K) >= 0
                   ? ip[m1]
                   : 0.0;
    }
  }
  // no barrier here: the first stage uses no table twiddles, and the first
  // exchange's barrier orders these stores before the second stage reads
  // them (last pass 302 -> 295 us in FP64)
  for (int x = tid; x < tw2_count(L1); x += NT) twl[x] = tw[ps.twL_off + x];
  f2_line<L1, HALVES>(v, t, ex + g * LP, twl);
  const int64_t n = pl.n, nf = a.nf, K = pl.K;
  if constexpr (G == 3) {
    const DevStats st = *stp;
    T2* cb = reinterpret_cast<T2*>(smem);  // [G][MR]: free once the last stage has read it
    double* pw = reinterpret_cast<double*>(outv) + m0 * L1;
    int* nill = const_cast<int*>(&stp->nill);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
      for (int j = r * (16 / NR); j < (r + 1) * (16 / NR); ++j)
        cb[g * MR + t + TL * j - r * MR] = v[f2_reg_of<L1>(j)];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const int mm = tid + NT * i;
        if (mm >= MR) continue;
        const int64_t m1 = r * MR + mm;
        const int64_t kout = fft2::crop(m0 + L0 * m1, n, nf, K);
        if (kout < 0) continue;
        const double ip = ipv[r * PPT + i];
        const T2 A = cb[mm], B = cb[MR + mm], B2 = cb[2 * MR + mm];
        double s6[6] = {(double)A.x * ip, (double)A.y * ip, (double)B.x * ip,
                        (double)B.y * ip, (double)B2.x * ip, (double)B2.y * ip};
        const int64_t q = kout - st.k_lo;
        const bool low = q >= 0 && q < st.nlow;
        if (low) {
          for (int c6 = 0; c6 < 6; ++c6) s6[c6] = lowfix[6 * q + c6];
          for (int pp = 1; pp < kLowParts; ++pp)
            for (int c6 = 0; c6 < 6; ++c6) s6[c6] += lowfix[pp * 6 * kLowMax + 6 * q + c6];
        }
        double p = ls_power(s6[0], s6[1], s6[2], s6[3], s6[4], s6[5], st, a.norm, a.fit_mean,
                            low ? 0.0 : a.dmin);
        if (kout == a.kzero) p = 0.0;
        else if (p != p) atomicAdd(nill, 1);
        pw[m1] = p;
      }
      if (r + 1 < NR) __syncthreads();
    }
  } else {
    double2* sums = reinterpret_cast<double2*>(outv) + m0 * L1;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t m1 = t + TL * j;
      if (fft2::crop(m0 + L0 * m1, n, nf, K) < 0) continue;
      const T2 A = v[f2_reg_of<L1>(j)];
      sums[m1] = make_double2((double)A.x * ipv[j], (double)A.y * ipv[j]);
    }
  }
}

// Last pass of a periodogram, one row m0 per workgroup of L1 / 16 threads
// that transform the row of the three grids one after another (the next
// grid's loads in flight meanwhile) and keep every result in registers:
// thread t then holds A, B and B2 of the same 16 modes m = m0 + L0 m1,
// m1 = t + (L1/16) j, and computes their power with no exchange.  The
// workgroup needs one exchange line of LDS, so that several fit a CU and one
// workgroup's loads overlap another's transform.  Power of mode m goes to
// out[m0 L1 + m1]; cropped modes are not written.
template <typename Real, int L1, int C, bool HALVES>
__global__ __launch_bounds__(L1 / 16, sizeof(Real) == 8 ? 1 : 2) void k_fft2_last_seq(Fft2Bufs<Real> b, FftPass ps,
                                                             Plan pl, CallArgs a,
                                                             const typename cplx<Real>::T* tw,
                                                             const double* iphi2,
                                                             const DevStats* stp,
                                                             const double* lowfix, double* pwout) {
  using T2 = typename cplx<Real>::T;
  using Lds = typename std::conditional<HALVES, Real, T2>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  if (stp->status != 0) return;
  constexpr int TL = L1 / 16, LP = fft2::line_pitch(L1);
  const int t = threadIdx.x;
  const int64_t L0 = ps.P;
  const int64_t m0 = xcd_remap(blockIdx.x, (int64_t)gridDim.x);
  Lds* ex = reinterpret_cast<Lds*>(smem);
  T2* twl = reinterpret_cast<T2*>(smem + (size_t)LP * sizeof(Lds));
  T2 va[16], vb[16], vc[16];
  auto load = [&](T2(&v)[16], int g) {
    const T2* in = b.mid[g] + m0 * L1;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = ld_stream(&in[t + q * TL]);
  };
  load(va, 0);
  load(vb, 1);
  for (int x = t; x < tw2_count(L1); x += TL) twl[x] = tw[ps.twL_off + x];
  __syncthreads();
  f2_line<L1, HALVES>(va, t, ex, twl);
  load(vc, 2);
  f2_line<L1, HALVES>(vb, t, ex, twl);
  f2_line<L1, HALVES>(vc, t, ex, twl);
  const int64_t n = pl.n, nf = a.nf, K = pl.K;
  const DevStats st = *stp;
  const double* ip = iphi2 + m0 * L1;
  double* pw = pwout + m0 * L1;
  int nan_count = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int64_t m1 = t + TL * j;
    const int64_t kout = fft2::crop(m0 + L0 * m1, n, nf, K);
    if (kout < 0) continue;
    const double iv = ip[m1];
    const int r = f2_reg_of<L1>(j);
    double s6[6] = {(double)va[r].x * iv, (double)va[r].y * iv, (double)vb[r].x * iv,
                    (double)vb[r].y * iv, (double)vc[r].x * iv, (double)vc[r].y * iv};
    const int64_t q = kout - st.k_lo;
    const bool low = q >= 0 && q < st.nlow;
    if (low) {
      for (int c6 = 0; c6 < 6; ++c6) s6[c6] = lowfix[6 * q + c6];
      for (int pp = 1; pp < kLowParts; ++pp)
        for (int c6 = 0; c6 < 6; ++c6) s6[c6] += lowfix[pp * 6 * kLowMax + 6 * q + c6];
    }
    double p = ls_power(s6[0], s6[1], s6[2], s6[3], s6[4], s6[5], st, a.norm, a.fit_mean,
                        low ? 0.0 : a.dmin);
    if (kout == a.kzero) p = 0.0;
    else if (p != p) ++nan_count;
    pw[m1] = p;
  }
  if (nan_count) atomicAdd(const_cast<int*>(&stp->nill), nan_count);
}

// Results of the last pass, [L0][L1] by (m0, m1), into frequency order:
// out[crop(m0 + L0 m1)] through TILE x TILE tiles in LDS (rows of the tile
// read along m1, written along m0, so both sides move whole lines; both
// streamed, as each element moves once).
template <typename V, int TILE>
__global__ __launch_bounds__(256) void k_fft2_out(const V* __restrict__ res, V* __restrict__ out,
                                                  int L0, int L1, int64_t n, int64_t nf, int64_t K,
                                                  const DevStats* st) {
  __shared__ V tile[TILE][TILE + 1];
  if (st->status != 0) return;
  constexpr int RS = 256 / TILE;
  const int64_t bid = xcd_remap(blockIdx.x, (int64_t)gridDim.x);
  const int nt1 = L1 / TILE;
  const int64_t tm1 = bid % nt1, tm0 = bid / nt1;
  // a tile whose modes all lie in the cropped band [nf - K, n - K) has
  // nothing to move (its modes grow with m1 by L0 across the tile)
  {
    const int64_t lo = tm0 * TILE + (int64_t)L0 * (tm1 * TILE);
    const int64_t hi = tm0 * TILE + TILE - 1 + (int64_t)L0 * (tm1 * TILE + TILE - 1);
    if (lo >= nf - K && hi < n - K) return;
  }
  const int tx = threadIdx.x % TILE, ty = threadIdx.x / TILE;
#pragma unroll
  for (int r = 0; r < TILE; r += RS) {
    const int64_t m0 = tm0 * TILE + r + ty;
    tile[r + ty][tx] = ld_stream(&res[m0 * L1 + tm1 * TILE + tx]);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < TILE; r += RS) {
    const int64_t m1 = tm1 * TILE + r + ty;
    const int64_t k = fft2::crop(tm0 * TILE + tx + (int64_t)L0 * m1, n, nf, K);
    if (k >= 0) st_stream(&out[k], tile[tx][r + ty]);
  }
}

// ============================================================================
// Direct sums: the three sums of every frequency evaluated term by term
// (Sec. 1, Eq. 1), O(N_d N_f), FP64 throughout; a check of the transform at
// any size and the paper's brute-force comparison.  A thread takes kDirF
// consecutive frequencies, a workgroup kDirThreads * kDirF; the points stream
// through LDS in chunks of kDirThreads, each staged once per workgroup:
// w^ y~, w^, the phase at the workgroup's first frequency fb and the phase
// step d = df (t - tau) (double-double, reduced mod 1), and exp(2 pi i d).  A
// thread's first phase is r_b + m d (m = its frequency offset, the product
// split exactly), reduced and turned into exp(2 pi i .) by sincospi; the
// next kDirF - 1 follow by multiplication with the step, and B2 uses the
// square of each.
// ============================================================================
constexpr int kDirF = 12;
constexpr int kDirThreads = 256;
struct DirPoint {
  double wy, wh, rb, dh, dl, sc, ss;
};

__global__ __launch_bounds__(kDirThreads) void k_direct(CallArgs a, Work w) {
  __shared__ DirPoint pts[kDirThreads];
  const DevStats st = *w.stats;
  if (st.status != 0) return;
  const int tid = threadIdx.x;
  const int64_t kb = (int64_t)blockIdx.x * kDirThreads * kDirF;
  const int m = tid * kDirF;
  const int64_t k0 = kb + m;
  // fb = f0 + kb df as a double-double
  double pp, pe;
  dd_two_prod((double)kb, a.df, pp, pe);
  double fbh, fbe;
  dd_two_sum(a.f0, pp, fbh, fbe);
  const double fbl = fbe + pe;
  const double invW = 1.0 / st.W;
  double acc[6][kDirF];
#pragma unroll
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int i = 0; i < kDirF; ++i) acc[q][i] = 0.0;
  for (int64_t j0 = 0; j0 < a.nd; j0 += kDirThreads) {
    const int64_t j = j0 + tid;
    if (j < a.nd) {
      DirPoint P;
      const double t = a.t[j];
      double wj = 1.0;
      if (a.dy) {
        const double dv = a.dy[j];
        wj = 1.0 / (dv * dv);
      }
      P.wh = wj * invW;
      P.wy = a.periodogram ? P.wh * (a.y[j] - st.ysub) : a.h[j];
      if (!a.periodogram) P.wh = 0.0;
      double th, tl;
      dd_two_sum(t, -st.tau, th, tl);
      // r_b = frac(fb (t - tau))
      double ah, al;
      dd_two_prod(fbh, th, ah, al);
      al = __builtin_fma(fbh, tl, al);
      al = __builtin_fma(fbl, th, al);
      double r = (ah - floor(ah)) + al;
      P.rb = r - rint(r);
      // d = frac(df (t - tau)) as a double-double
      double dh, dl;
      dd_two_prod(a.df, th, dh, dl);
      dl = __builtin_fma(a.df, tl, dl);
      const double df0 = dh - floor(dh);
      double d2h, d2l;
      dd_two_sum(df0, dl, d2h, d2l);
      P.dh = d2h;
      P.dl = d2l;
      sincospi(2.0 * (d2h + d2l), &P.ss, &P.sc);
      pts[tid] = P;
    }
    __syncthreads();
    const int cnt = (int)(a.nd - j0 < kDirThreads ? a.nd - j0 : kDirThreads);
    for (int i = 0; i < cnt; ++i) {
      const DirPoint P = pts[i];
      // phase of frequency k0: r_b + m d (mod 1)
      double mp, me;
      dd_two_prod((double)m, P.dh, mp, me);
      double ph = (mp - floor(mp)) + P.rb;
      ph += __builtin_fma((double)m, P.dl, me);
      ph -= rint(ph);
      double zs, zc;
      sincospi(2.0 * ph, &zs, &zc);
#pragma unroll
      for (int f = 0; f < kDirF; ++f) {
        acc[0][f] = __builtin_fma(P.wy, zc, acc[0][f]);
        acc[1][f] = __builtin_fma(P.wy, zs, acc[1][f]);
        acc[2][f] = __builtin_fma(P.wh, zc, acc[2][f]);
        acc[3][f] = __builtin_fma(P.wh, zs, acc[3][f]);
        const double c2 = __builtin_fma(zc, zc, -zs * zs);
        const double s2 = 2.0 * zc * zs;
        acc[4][f] = __builtin_fma(P.wh, c2, acc[4][f]);
        acc[5][f] = __builtin_fma(P.wh, s2, acc[5][f]);
        const double nc = __builtin_fma(zc, P.sc, -zs * P.ss);
        zs = __builtin_fma(zc, P.ss, zs * P.sc);
        zc = nc;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int f = 0; f < kDirF; ++f) {
    const int64_t k = k0 + f;
    if (k >= a.nf) break;
    if (a.periodogram) {
      double pw = ls_power(acc[0][f], acc[1][f], acc[2][f], acc[3][f], acc[4][f], acc[5][f], st,
                           a.norm, a.fit_mean, 0.0);
      if (k == a.kzero) pw = 0.0;
      else if (pw != pw) atomicAdd(&w.stats->nill, 1);
      a.power[k] = pw;
    } else {
      a.sums[2 * k] = acc[0][f];
      a.sums[2 * k + 1] = acc[1][f];
    }
  }
}

// ============================================================================
// Host launchers
// ============================================================================
static inline unsigned grid_for(int64_t work, int64_t cap) {
  int64_t b = (work + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

// Dynamic LDS above the default 64 KB of a workgroup must be allowed per
// kernel (the big FFT passes use up to kLdsBig).
static void big_lds(const void* kern, size_t bytes) {
  // once per kernel (the largest request so far), so that a call captured
  // into a graph after a first uncaptured one makes no attribute call
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  if (bytes <= 65536) return;
  std::lock_guard<std::mutex> lk(mu);
  size_t& have = done[kern];
  if (have >= bytes) return;
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
      hipSuccess)
    have = bytes;
  else
    (void)hipGetLastError();  // the launch then reports the refusal itself
}

hipError_t launch_phihat2(double* iphi2, const double* inv_phihat, int L0, int L1, int64_t n,
                          int64_t nf, int64_t K, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_phihat2, dim3(grid_for(n, 1 << 30)), dim3(kThreads), 0, s, iphi2,
                     inv_phihat, L0, L1, n, nf, K);
  return hipGetLastError();
}

hipError_t launch_phihat(double* inv_phihat, int64_t K, double w, double n, const double* z,
                         const double* gphi, int q, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_phihat, dim3(grid_for(K + 1, 1 << 30)), dim3(kThreads), 0, s, inv_phihat,
                     K, w, n, z, gphi, q);
  return hipGetLastError();
}

// Statistics of the call (k_stats + k_stats_final into w.stats).
static void enqueue_stats(const CallArgs& a, const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_stats, dim3(kStatsBlocks), dim3(kThreads), 0, s, a, w);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kThreads), 0, s, a, w, kStatsBlocks);
}

// Binning: the sorted fast path, then the counting sort, whose kernels exit
// at once unless the fast path found a descent.
static void enqueue_bins(const CallArgs& a, const Plan& p, const Work& w, hipStream_t s) {
  const int64_t nbt = (a.nd > p.nbins + 1 ? a.nd : p.nbins + 1);
  hipLaunchKernelGGL(k_bins_sorted, dim3(grid_for(nbt, 1 << 20)), dim3(kThreads), 0, s, a, p, w);
  const unsigned sort_blocks = grid_for(a.nd > p.nbins ? a.nd : p.nbins, 512);
  hipLaunchKernelGGL(k_sort_hist, dim3(sort_blocks), dim3(kThreads), 0, s, a, p, w);
  const int64_t nchunks = (p.nbins + 1 + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan1, dim3((unsigned)nchunks), dim3(kThreads), 0, s, p, w);
  hipLaunchKernelGGL(k_scan3, dim3((unsigned)nchunks), dim3(kThreads), 0, s, p, w);
  hipLaunchKernelGGL(k_sort_scatter, dim3(sort_blocks), dim3(kThreads), 0, s, a, p, w);
}

// Reproducible binning (see k_det_keys).
static void enqueue_det_bins(const CallArgs& a, const Plan& p, const Work& w, hipStream_t s) {
  const int64_t nk = det_keys(a.nd);
  const unsigned g = grid_for(nk, 1 << 16);
  hipLaunchKernelGGL(k_det_keys, dim3(g), dim3(kThreads), 0, s, a, p, w, nk);
  for (int64_t k = 2; k <= nk; k <<= 1)
    for (int64_t jj = k >> 1; jj > 0; jj >>= 1)
      hipLaunchKernelGGL(k_det_bitonic, dim3(g), dim3(kThreads), 0, s, w, nk, k, jj);
  const int64_t nbt = (a.nd > p.nbins + 1 ? a.nd : p.nbins + 1);
  hipLaunchKernelGGL(k_det_gather, dim3(grid_for(nbt, 1 << 16)), dim3(kThreads), 0, s, a, p, w);
}

// Direct sums near f = 0 into w.lowfix.
static void enqueue_lowfreq(const CallArgs& a, const Work& w, hipStream_t s) {
  const unsigned lb = grid_for(a.nd, kLowBlocks);
  hipLaunchKernelGGL(k_lowfreq, dim3(lb), dim3(kThreads), 0, s, a, w);
  hipLaunchKernelGGL(k_lowfreq_final, dim3(kLowParts), dim3(kLowFinalThreads), 0, s, a, w,
                     (int)lb);
}

// One first/middle FFT pass over ng grids of b.
template <typename Real>
static void enqueue_pass(const FftPass& ps, const PassBufs<Real>& b, int ng, const Work& w,
                         hipStream_t st) {
  using T2 = typename cplx<Real>::T;
  constexpr bool f64 = sizeof(Real) == 8;
  constexpr int EMID = f64 ? kEmid64 : kEmid32;
  constexpr int EBIG = f64 ? kEbig64 : kEbig32;
  const T2* tw = reinterpret_cast<const T2*>(w.tw);
  const int64_t nblk = ps.P * ((ps.S + ps.C - 1) / ps.C);
  const int ntw = ps.big ? tw2_count(ps.L) : ps.L;
  const size_t lds = sizeof(T2) * (size_t)(ps.L * ps.C + ntw) + (size_t)ps.L + 16;
  if (ps.big) {
    auto kern = k_fft_pass<Real, EBIG, kThreadsBig, true>;
    big_lds(reinterpret_cast<const void*>(kern), lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk, ng), dim3(kThreadsBig), lds, st, b, ps, tw,
                       w.stats);
  } else {
    hipLaunchKernelGGL((k_fft_pass<Real, EMID, kThreads, false>), dim3((unsigned)nblk, ng),
                       dim3(kThreads), lds, st, b, ps, tw, w.stats);
  }
}

// The last FFT pass over G grids of b: with power (G = 3, or G = 1 for a
// series sharing its weights), or the complex sums (G = 1).
template <typename Real>
static void enqueue_last(const CallArgs& a, const Plan& p, const PassBufs<Real>& b, int G,
                         const Work& w, hipStream_t s) {
  using T2 = typename cplx<Real>::T;
  constexpr bool f64 = sizeof(Real) == 8;
  constexpr int ELAST = f64 ? kElast64 : kElast32;
  constexpr int EBIG = f64 ? kEbig64 : kEbig32;
  constexpr int NTL = last_threads<Real>();
  const T2* tw = reinterpret_cast<const T2*>(w.tw);
  const FftPass& ps = p.pass[p.npass - 1];
  const int64_t nblk = (ps.P + ps.C - 1) / ps.C;
  const int ntw = ps.big ? tw2_count(ps.L) : ps.L;
  const size_t lds = sizeof(T2) * (size_t)(ps.L * last_pitch(G * ps.C) + ntw);
  const dim3 grid((unsigned)nblk);
  const auto* ip = w.inv_phihat;
  if (a.nser > 0) {
    // a group of series sharing their weights (a plan made for three grids,
    // so D L <= ELAST / 3): grid g holds series g's A sums
    if (ps.big) {
      auto kern = k_fft_last_ser<Real, 1, EBIG, kThreadsBig, true>;
      big_lds(reinterpret_cast<const void*>(kern), lds);
      hipLaunchKernelGGL(kern, grid, dim3(kThreadsBig), lds, s, b, ps, p, a, tw, ip, w.stats,
                         w.lowfix);
    } else if (G == 3) {
      hipLaunchKernelGGL((k_fft_last_ser<Real, 3, ELAST, NTL, false>), grid, dim3(NTL), lds, s,
                         b, ps, p, a, tw, ip, w.stats, w.lowfix);
    } else if (G == 2) {
      hipLaunchKernelGGL((k_fft_last_ser<Real, 2, 2 * (ELAST / 3), NTL, false>), grid, dim3(NTL),
                         lds, s, b, ps, p, a, tw, ip, w.stats, w.lowfix);
    } else {
      hipLaunchKernelGGL((k_fft_last_ser<Real, 1, ELAST / 3, NTL, false>), grid, dim3(NTL), lds,
                         s, b, ps, p, a, tw, ip, w.stats, w.lowfix);
    }
  } else if (ps.big) {
    auto kern = G == 3 ? k_fft_last<Real, 3, EBIG, kThreadsBig, true>
                       : k_fft_last<Real, 1, EBIG, kThreadsBig, true>;
    big_lds(reinterpret_cast<const void*>(kern), lds);
    hipLaunchKernelGGL(kern, grid, dim3(kThreadsBig), lds, s, b, ps, p, a, tw, ip, w.stats,
                       w.lowfix);
  } else if (G == 3) {
    hipLaunchKernelGGL((k_fft_last<Real, 3, ELAST, NTL, false>), grid, dim3(NTL), lds, s, b, ps,
                       p, a, tw, ip, w.stats, w.lowfix);
  } else if (ps.C * ps.L <= ELAST / 3) {
    // one grid of a plan made for three (the weight-only sums): the
    // third-size instance holds a third of the registers
    hipLaunchKernelGGL((k_fft_last<Real, 1, ELAST / 3, NTL, false>), grid, dim3(NTL), lds, s, b,
                       ps, p, a, tw, ip, w.stats, w.lowfix);
  } else {
    hipLaunchKernelGGL((k_fft_last<Real, 1, ELAST, NTL, false>), grid, dim3(NTL), lds, s, b, ps,
                       p, a, tw, ip, w.stats, w.lowfix);
  }
}

// Grids g0 .. g0+ng-1 of w through every pass but the last: the first pass
// in place (row flags of their geometry: grid grid_2f is of geometry 2f, the
// others of geometry f), the middle ones alternating with the second grid
// set.  in[i] receives where grid g0+i ends up.
template <typename Real>
static void enqueue_passes(const Plan& p, const Work& w, int g0, int ng, int grid_2f,
                           hipStream_t s, typename cplx<Real>::T** in) {
  using T2 = typename cplx<Real>::T;
  T2* cur[3];
  T2* alt[3];
  for (int i = 0; i < ng; ++i) {
    cur[i] = reinterpret_cast<T2*>(w.grid[g0 + i]);
    alt[i] = reinterpret_cast<T2*>(w.grid2[g0 + i]);
  }
  for (int ip = 0; ip + 1 < p.npass; ++ip) {
    PassBufs<Real> b;
    for (int i = 0; i < 3; ++i) {
      const int j = i < ng ? i : ng - 1;
      b.in[i] = cur[j];
      b.out[i] = ip == 0 ? cur[j] : alt[j];
      b.rowflag[i] = ip == 0 ? (g0 + j == grid_2f ? w.rowflag_2f : w.rowflag_f) : nullptr;
    }
    enqueue_pass<Real>(p.pass[ip], b, ng, w, s);
    if (ip > 0)
      for (int i = 0; i < ng; ++i) {
        T2* tmp = cur[i];
        cur[i] = alt[i];
        alt[i] = tmp;
      }
  }
  for (int i = 0; i < ng; ++i) in[i] = cur[i];
}

// First pass of the two-pass FFT over ng grids (b.grid[0 .. ng-1]).
template <typename Real, int L0, int C>
static void enqueue_fft2_first_l(const Plan& p, const Fft2Bufs<Real>& b, int ng, const Work& w,
                                 hipStream_t st) {
  using T2 = typename cplx<Real>::T;
  constexpr bool H = sizeof(Real) == 8;
  const FftPass& ps = p.pass[0];
  auto kern = k_fft2_first<Real, L0, C, H>;
  const size_t lds = f2_first_lds<Real>(L0, C, H);
  big_lds(reinterpret_cast<const void*>(kern), lds);
  hipLaunchKernelGGL(kern, dim3((unsigned)(ps.S / C), ng), dim3(C * L0 / 16), lds, st, b, ps,
                     reinterpret_cast<const T2*>(w.tw), w.stats);
}

template <typename Real>
static void enqueue_fft2_first(const Plan& p, const Fft2Bufs<Real>& b, int ng, const Work& w,
                               hipStream_t st) {
  const int L0 = p.pass[0].L, C = p.pass[0].C;
  if (L0 == 2048 && C == 8) enqueue_fft2_first_l<Real, 2048, 8>(p, b, ng, w, st);
  else if (L0 == 2048) enqueue_fft2_first_l<Real, 2048, 4>(p, b, ng, w, st);
  else if (L0 == 4096 && C == 4) enqueue_fft2_first_l<Real, 4096, 4>(p, b, ng, w, st);
  else if (L0 == 4096) enqueue_fft2_first_l<Real, 4096, 2>(p, b, ng, w, st);
  else enqueue_fft2_first_l<Real, 8192, 2>(p, b, ng, w, st);
}

template <typename Real, int L1, int G>
static void enqueue_fft2_last_l(const CallArgs& a, const Plan& p, const Fft2Bufs<Real>& b,
                                const Work& w, hipStream_t st) {
  using T2 = typename cplx<Real>::T;
  constexpr bool H = sizeof(Real) == 8;
  const int L0 = p.pass[0].L;
  const int C = p.pass[0].C;
  const FftPass& ps = p.pass[1];
  const size_t lds = f2_last_lds<Real>(L1, G, H);
  const T2* tw = reinterpret_cast<const T2*>(w.tw);
  const double* lowfix = G == 3 ? w.lowfix : nullptr;
#define MILS_F2_LAST(CC)                                                                         \
  if (G == 3 && !H) {                                                                          \
    auto kern = k_fft2_last_seq<Real, L1, CC, H>;                                              \
    const size_t lds3 = f2_last_seq_lds<Real>(L1, H);                                          \
    big_lds(reinterpret_cast<const void*>(kern), lds3);                                        \
    hipLaunchKernelGGL(kern, dim3((unsigned)L0), dim3(L1 / 16), lds3, st, b, ps, p, a, tw,      \
                       w.inv_phihat2, w.stats, lowfix, reinterpret_cast<double*>(w.f2out));    \
  } else {                                                                                     \
    auto kern = k_fft2_last<Real, L1, G, CC, H>;                                               \
    big_lds(reinterpret_cast<const void*>(kern), lds);                                         \
    hipLaunchKernelGGL(kern, dim3((unsigned)L0), dim3(G * L1 / 16), lds, st, b, ps, p, a, tw,   \
                       w.inv_phihat2, w.stats, lowfix, w.f2out);                               \
  }
  if (C == 8) MILS_F2_LAST(8)
  else if (C == 4) MILS_F2_LAST(4)
  else MILS_F2_LAST(2)
#undef MILS_F2_LAST
}

// The tiled transpose of the last pass's results into frequency order.
static void enqueue_fft2_out(const CallArgs& a, const Plan& p, int G, const Work& w,
                             hipStream_t st) {
  const int L0 = p.pass[0].L, L1 = p.pass[1].L;
  const int64_t nblk = (int64_t)(L0 / (G == 3 ? 64 : 32)) * (L1 / (G == 3 ? 64 : 32));
  if (G == 3)
    hipLaunchKernelGGL((k_fft2_out<double, 64>), dim3((unsigned)nblk), dim3(256), 0, st,
                       reinterpret_cast<const double*>(w.f2out), a.power, L0, L1, p.n, a.nf, p.K,
                       w.stats);
  else
    hipLaunchKernelGGL((k_fft2_out<double2, 32>), dim3((unsigned)nblk), dim3(256), 0, st,
                       reinterpret_cast<const double2*>(w.f2out),
                       reinterpret_cast<double2*>(a.sums), L0, L1, p.n, a.nf, p.K, w.stats);
}

template <typename Real>
static void enqueue_fft2_last(const CallArgs& a, const Plan& p, const Fft2Bufs<Real>& b, int G,
                              const Work& w, hipStream_t st) {
  const int L1 = p.pass[1].L;
  if (G == 3) {
    if (L1 == 2048) enqueue_fft2_last_l<Real, 2048, 3>(a, p, b, w, st);
    else enqueue_fft2_last_l<Real, 4096, 3>(a, p, b, w, st);
  } else {
    if (L1 == 2048) enqueue_fft2_last_l<Real, 2048, 1>(a, p, b, w, st);
    else if (L1 == 4096) enqueue_fft2_last_l<Real, 4096, 1>(a, p, b, w, st);
    else enqueue_fft2_last_l<Real, 8192, 1>(a, p, b, w, st);
  }
}

template <typename Real>
static hipError_t launch_path_t(const CallArgs& a, const Plan& p, const Work& w, hipStream_t s,
                                const StageHook* hook, const AuxStream* aux) {
  using T2 = typename cplx<Real>::T;
  const int G = a.periodogram ? 3 : 1;
  // The periodogram forks after binning: the 2f geometry (row flags, spread,
  // first FFT pass of its grid) and the direct sums near f = 0 run on the
  // auxiliary stream, beside the f geometry, and join before the second pass.
  const bool fork = a.periodogram && aux != nullptr;
  hipStream_t s2 = fork ? aux->s : s;
  auto mark = [&](int stage, int begin, hipStream_t st) {
    if (hook) hook->fn(hook->ud, stage, begin, st);
  };
  mark(kStageStats, 1, s);
  enqueue_stats(a, w, s);
  mark(kStageStats, 0, s);
  mark(kStageBin, 1, s);
  if (a.deterministic) enqueue_det_bins(a, p, w, s);
  else enqueue_bins(a, p, w, s);
  mark(kStageBin, 0, s);
  const int nd = (int)a.nd;
  // two-pass plans classify the rows of both geometries before the fork:
  // beside the other branch's persistent spread, a one-workgroup launch
  // waits long for a free CU
  const bool rows_first = p.fft2 && a.periodogram;
  if (rows_first) {
    mark(kStageRows, 1, s);
    enqueue_row_class(p, w, nd, 0, 2, s);
    mark(kStageRows, 0, s);
  }
  if (fork) {
    hipError_t e = hipEventRecord(aux->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s2, aux->fork, 0);
    if (e != hipSuccess) return e;
  }

  const int64_t ntiles = (p.S1 / p.T) * p.nrows;
  const unsigned sgrid = (unsigned)(ntiles < kSpreadGrid ? ntiles : kSpreadGrid);
  // The f geometry (row classes, spread and then the first FFT pass of its
  // two grids) is the longer branch: it is launched (and captured) first.
  mark(kStageSpreadF, 1, s);
  if (!rows_first)
    enqueue_row_class(p, w, nd, 0, 1, s);
  if (a.periodogram && a.deterministic)
    hipLaunchKernelGGL((k_spread_rows<Real, 1, 2, true>), dim3(sgrid), dim3(kThreads), 0, s, a, p,
                       w, 0, w.act_rows_f, 0);
  else if (a.periodogram)
    hipLaunchKernelGGL((k_spread_rows<Real, 1, 2>), dim3(sgrid), dim3(kThreads), 0, s, a, p, w, 0,
                       w.act_rows_f, 0);
  else
    hipLaunchKernelGGL((k_spread_rows<Real, 1, 1>), dim3(sgrid), dim3(kThreads), 0, s, a, p, w, 0,
                       w.act_rows_f, 0);
  mark(kStageSpreadF, 0, s);
  if (a.periodogram && !p.fft2) {
    mark(kStageLow, 1, s2);
    enqueue_lowfreq(a, w, s2);
    mark(kStageLow, 0, s2);
  }
  if (a.periodogram) {
    mark(kStageSpread2F, 1, s2);
    if (!rows_first)
      enqueue_row_class(p, w, nd, 1, 1, s2);
    if (a.deterministic)
      hipLaunchKernelGGL((k_spread_rows<Real, 2, 1, true>), dim3(sgrid), dim3(kThreads), 0, s2, a,
                         p, w, 2, w.act_rows_2f, 1);
    else
      hipLaunchKernelGGL((k_spread_rows<Real, 2, 1>), dim3(sgrid), dim3(kThreads), 0, s2, a, p, w,
                         2, w.act_rows_2f, 1);
    mark(kStageSpread2F, 0, s2);
  }
  if (p.fft2) {
    // two-pass register-tile FFT: the first pass of each geometry's grids on
    // its branch, then (joined) the last pass and the transpose
    Fft2Bufs<Real> b;
    for (int g = 0; g < 3; ++g) {
      b.grid[g] = reinterpret_cast<T2*>(w.grid[g < G ? g : 0]);
      b.mid[g] = reinterpret_cast<T2*>(w.grid2[g < G ? g : 0]);
      b.rowflag[g] = g == 2 ? w.rowflag_2f : w.rowflag_f;
    }
    if (fork) {
      // both spreads first (the first pass fills every CU and would starve
      // the other branch's small kernels), then the first pass of all three
      // grids in one launch beside the direct sums near f = 0
      hipError_t e = hipEventRecord(aux->mid, s2);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, aux->mid, 0);
      if (e != hipSuccess) return e;
      mark(kStagePass0, 1, s);
      enqueue_fft2_first<Real>(p, b, 3, w, s);
      mark(kStagePass0, 0, s);
      mark(kStageLow, 1, s2);
      enqueue_lowfreq(a, w, s2);
      mark(kStageLow, 0, s2);
      e = hipEventRecord(aux->join, s2);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, aux->join, 0);
      if (e != hipSuccess) return e;
    } else {
      if (a.periodogram) {
        mark(kStageLow, 1, s);
        enqueue_lowfreq(a, w, s);
        mark(kStageLow, 0, s);
      }
      mark(kStagePass0, 1, s);
      enqueue_fft2_first<Real>(p, b, G, w, s);
      mark(kStagePass0, 0, s);
    }
    mark(kStageLast, 1, s);
    enqueue_fft2_last<Real>(a, p, b, G, w, s);
    mark(kStageLast, 0, s);
    mark(kStageOut, 1, s);
    enqueue_fft2_out(a, p, G, w, s);
    mark(kStageOut, 0, s);
    return hipGetLastError();
  }
  // passes 0 .. npass-2; launch over grids [g0, g0 + ng) of the current set
  T2* cur[3];
  T2* alt[3];
  for (int g = 0; g < 3; ++g) {
    cur[g] = reinterpret_cast<T2*>(w.grid[g]);
    alt[g] = reinterpret_cast<T2*>(w.grid2[g]);
  }
  auto pass = [&](int ip, int g0, int ng, hipStream_t st) {
    PassBufs<Real> b;
    for (int i = 0; i < 3; ++i) {
      const int g = g0 + i < 3 ? g0 + i : 2;
      b.in[i] = cur[g];
      b.out[i] = (ip == 0) ? cur[g] : alt[g];
      b.rowflag[i] = (ip == 0) ? (g == 2 ? w.rowflag_2f : w.rowflag_f) : nullptr;
    }
    enqueue_pass<Real>(p.pass[ip], b, ng, w, st);
  };
  if (p.npass >= 2) {
    if (fork) {
      mark(kStagePass0, 1, s);
      pass(0, 0, 2, s);   // f grids
      mark(kStagePass0, 0, s);
      mark(kStagePass0, 1, s2);
      pass(0, 2, 1, s2);  // 2f grid
      mark(kStagePass0, 0, s2);
    } else {
      mark(kStagePass0, 1, s);
      pass(0, 0, G, s);
      mark(kStagePass0, 0, s);
    }
  }
  if (fork) {
    hipError_t e = hipEventRecord(aux->join, s2);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, aux->join, 0);
    if (e != hipSuccess) return e;
  }
  for (int ip = 1; ip + 1 < p.npass; ++ip) {
    mark(kStagePass0 + ip, 1, s);
    pass(ip, 0, G, s);
    mark(kStagePass0 + ip, 0, s);
    for (int g = 0; g < 3; ++g) {
      T2* tmp = cur[g];
      cur[g] = alt[g];
      alt[g] = tmp;
    }
  }
  {
    PassBufs<Real> b;
    for (int g = 0; g < 3; ++g) {
      b.in[g] = cur[g];
      b.out[g] = nullptr;
      b.rowflag[g] = nullptr;
    }
    mark(kStageLast, 1, s);
    enqueue_last<Real>(a, p, b, G, w, s);
    mark(kStageLast, 0, s);
  }
  return hipGetLastError();
}

// Every launch sequence below reports hipGetLastError() after its launches;
// it first discards the calling thread's last error, which an earlier,
// already handled failure (a refused allocation) may have left set and
// which would otherwise be taken for a failed launch.
hipError_t launch_path(const CallArgs& a, const Plan& p, const Work& w, hipStream_t s,
                       const StageHook* hook, const AuxStream* aux) {
  (void)hipGetLastError();
  if (p.prec == 1) return launch_path_t<float>(a, p, w, s, hook, aux);
  return launch_path_t<double>(a, p, w, s, hook, aux);
}

// ============================================================================
// Series sharing their observation times and weights (the batched mode for
// shared times): B (geometry f) and B2 (geometry 2f) depend on t and the
// weights only, so they are computed once, and each series adds the sum A
// through one grid.
// ============================================================================
template <typename Real>
static hipError_t launch_weight_sums_t(const CallArgs& aw, const Plan& p, const Work& w,
                                       double* bsum_b, double* bsum_b2, hipStream_t s) {
  using T2 = typename cplx<Real>::T;
  enqueue_stats(aw, w, s);
  enqueue_bins(aw, p, w, s);
  const int64_t ntiles = (p.S1 / p.T) * p.nrows;
  const unsigned sgrid = (unsigned)(ntiles < kSpreadGrid ? ntiles : kSpreadGrid);
  const int nd = (int)aw.nd;
  enqueue_row_class(p, w, nd, 0, 2, s);
  hipLaunchKernelGGL((k_spread_rows<Real, 1, 1>), dim3(sgrid), dim3(kThreads), 0, s, aw, p, w, 1,
                     w.act_rows_f, 0);
  hipLaunchKernelGGL((k_spread_rows<Real, 2, 1>), dim3(sgrid), dim3(kThreads), 0, s, aw, p, w, 2,
                     w.act_rows_2f, 1);
  T2* in[2];
  enqueue_passes<Real>(p, w, 1, 2, 2, s, in);
  CallArgs as = aw;
  as.periodogram = 0;  // the last pass writes the deconvolved sums
  for (int i = 0; i < 2; ++i) {
    PassBufs<Real> b;
    for (int g = 0; g < 3; ++g) {
      b.in[g] = in[i];
      b.out[g] = nullptr;
      b.rowflag[g] = nullptr;
    }
    as.sums = i == 0 ? bsum_b : bsum_b2;
    enqueue_last<Real>(as, p, b, 1, w, s);
  }
  return hipGetLastError();
}

template <typename Real>
static hipError_t launch_series_group_t(const CallArgs& a, const Plan& p, const Work& w,
                                        const SeriesGroup& sg, hipStream_t s) {
  using T2 = typename cplx<Real>::T;
  const int64_t ntiles = (p.S1 / p.T) * p.nrows;
  const unsigned sgrid = (unsigned)(ntiles < kSpreadGrid ? ntiles : kSpreadGrid);
  CallArgs al = a;
  al.nser = sg.m;
  for (int g = 0; g < sg.m; ++g) {
    // statistics, binning (only when the points must be sorted: the sorted
    // copy of y is the series' own; otherwise the weights-only call's bins
    // hold), direct sums near f = 0, and the A spread into grid g
    CallArgs ag = a;
    ag.y = sg.y[g];
    Work wg = w;
    wg.stats = sg.stats[g];
    wg.lowfix = sg.lowfix[g];
    enqueue_stats(ag, wg, s);
    if (sg.need_sort) enqueue_bins(ag, p, wg, s);
    enqueue_lowfreq(ag, wg, s);
    hipLaunchKernelGGL((k_spread_rows<Real, 1, 1>), dim3(sgrid), dim3(kThreads), 0, s, ag, p, wg,
                       g, w.act_rows_f, 0);
    al.spow[g] = sg.power[g];
    al.sst[g] = sg.stats[g];
    al.slow[g] = sg.lowfix[g];
  }
  T2* in[3];
  enqueue_passes<Real>(p, w, 0, sg.m, -1, s, in);
  PassBufs<Real> b;
  for (int g = 0; g < 3; ++g) {
    b.in[g] = in[g < sg.m ? g : sg.m - 1];
    b.out[g] = nullptr;
    b.rowflag[g] = nullptr;
  }
  enqueue_last<Real>(al, p, b, sg.m, w, s);
  return hipGetLastError();
}

hipError_t launch_weight_sums(const CallArgs& aw, const Plan& p, const Work& w, double* bsum_b,
                              double* bsum_b2, hipStream_t s) {
  (void)hipGetLastError();
  if (p.prec == 1) return launch_weight_sums_t<float>(aw, p, w, bsum_b, bsum_b2, s);
  return launch_weight_sums_t<double>(aw, p, w, bsum_b, bsum_b2, s);
}

hipError_t launch_series_group(const CallArgs& a, const Plan& p, const Work& w,
                               const SeriesGroup& sg, hipStream_t s) {
  if (sg.m < 1 || sg.m > 3) return hipErrorInvalidValue;
  (void)hipGetLastError();
  if (p.prec == 1) return launch_series_group_t<float>(a, p, w, sg, s);
  return launch_series_group_t<double>(a, p, w, sg, s);
}

hipError_t launch_direct(const CallArgs& a, const Work& w, hipStream_t s) {
  (void)hipGetLastError();
  enqueue_stats(a, w, s);
  const int64_t per = (int64_t)kDirThreads * kDirF;
  const int64_t nb = (a.nf + per - 1) / per;
  hipLaunchKernelGGL(k_direct, dim3((unsigned)nb), dim3(kDirThreads), 0, s, a, w);
  return hipGetLastError();
}

}  // namespace mils
