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

#include "device_math.h"
#include "fft_core.h"
#include "kernels.h"
#include "mils_internal.h"

namespace mils {

// ============================================================================
// Statistics: weighted mean/variance (merged Welford moments), time range,
// sortedness and validity.  One launch; the last block to finish combines the
// per-block partials and writes the scalars of the call.
// ============================================================================
struct Moments {
  double W, mu, M2;
};

__device__ __forceinline__ void moments_merge(Moments& a, double Wb, double mub, double M2b) {
  double W = a.W + Wb;
  if (W == 0.0) return;
  double d = mub - a.mu;
  double fb = Wb / W;
  a.mu += d * fb;
  a.M2 += M2b + d * d * a.W * fb;
  a.W = W;
}

__global__ __launch_bounds__(kThreads) void k_stats(CallArgs a, Work w) {
  __shared__ double sW[kThreads], sMu[kThreads], sM2[kThreads], sLo[kThreads], sHi[kThreads];
  __shared__ int sBad[kThreads], sUns[kThreads];
  __shared__ bool amLast;
  const int tid = threadIdx.x;
  Moments m = {0.0, 0.0, 0.0};
  double lo = INFINITY, hi = -INFINITY;
  int bad = 0, uns = 0;
  const double* yv = a.periodogram ? a.y : a.h;
  for (int64_t j = (int64_t)blockIdx.x * kThreads + tid; j < a.nd; j += (int64_t)gridDim.x * kThreads) {
    double t = a.t[j];
    double y = yv[j];
    double wj = 1.0;
    if (a.dy) {
      double d = a.dy[j];
      if (!(d > 0.0) || !isfinite(d)) bad = 1;
      wj = 1.0 / (d * d);
    }
    if (!isfinite(t) || !isfinite(y) || !isfinite(wj)) bad = 1;
    if (j > 0 && t < a.t[j - 1]) uns = 1;
    lo = fmin(lo, t);
    hi = fmax(hi, t);
    moments_merge(m, wj, y, 0.0);
  }
  sW[tid] = m.W;
  sMu[tid] = m.mu;
  sM2[tid] = m.M2;
  sLo[tid] = lo;
  sHi[tid] = hi;
  sBad[tid] = bad;
  sUns[tid] = uns;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      Moments x = {sW[tid], sMu[tid], sM2[tid]};
      moments_merge(x, sW[tid + s], sMu[tid + s], sM2[tid + s]);
      sW[tid] = x.W;
      sMu[tid] = x.mu;
      sM2[tid] = x.M2;
      sLo[tid] = fmin(sLo[tid], sLo[tid + s]);
      sHi[tid] = fmax(sHi[tid], sHi[tid + s]);
      sBad[tid] |= sBad[tid + s];
      sUns[tid] |= sUns[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* p = w.partials + 8 * blockIdx.x;
    p[0] = sW[0];
    p[1] = sMu[0];
    p[2] = sM2[0];
    p[3] = sLo[0];
    p[4] = sHi[0];
    p[5] = (double)sBad[0];
    p[6] = (double)sUns[0];
    __threadfence();
    unsigned int prev = atomicAdd(&w.stats->done, 1u);
    amLast = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!amLast) return;
  __threadfence();
  // final combine over the per-block partials
  m = {0.0, 0.0, 0.0};
  lo = INFINITY;
  hi = -INFINITY;
  bad = 0;
  uns = 0;
  for (int b = tid; b < (int)gridDim.x; b += kThreads) {
    const volatile double* p = w.partials + 8 * b;
    moments_merge(m, p[0], p[1], p[2]);
    lo = fmin(lo, p[3]);
    hi = fmax(hi, p[4]);
    bad |= (p[5] != 0.0);
    uns |= (p[6] != 0.0);
  }
  sW[tid] = m.W;
  sMu[tid] = m.mu;
  sM2[tid] = m.M2;
  sLo[tid] = lo;
  sHi[tid] = hi;
  sBad[tid] = bad;
  sUns[tid] = uns;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      Moments x = {sW[tid], sMu[tid], sM2[tid]};
      moments_merge(x, sW[tid + s], sMu[tid + s], sM2[tid + s]);
      sW[tid] = x.W;
      sMu[tid] = x.mu;
      sM2[tid] = x.M2;
      sLo[tid] = fmin(sLo[tid], sLo[tid + s]);
      sHi[tid] = fmax(sHi[tid], sHi[tid + s]);
      sBad[tid] |= sBad[tid + s];
      sUns[tid] |= sUns[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    DevStats* st = w.stats;
    st->W = sW[0];
    st->mu = sMu[0];
    st->M2 = sM2[0];
    st->tmin = sLo[0];
    st->tmax = sHi[0];
    st->invalid = sBad[0];
    st->unsorted = sUns[0];
    st->need_sort = sUns[0];
    st->tau = a.periodogram ? sLo[0] : 0.0;
    double W = sW[0];
    st->ysub = a.center ? sMu[0] : 0.0;
    st->Ybar = a.center ? 0.0 : sMu[0];
    double YY = sM2[0] / W;
    if (!a.fit_mean && !a.center) YY += sMu[0] * sMu[0];
    st->YY = YY;
    int status = 0;
    if (sBad[0]) status = -1;
    else if (a.periodogram && !(YY > 0.0)) status = -2;
    st->status = status;
    st->done = 0u;
  }
}

// ============================================================================
// Binning.  bin_start[b] = index of the first point (in the order the spread
// reads them) whose cell lies in bin b or later; bin_start[nbins] = nd.
// ============================================================================
__device__ __forceinline__ int point_bin(double t, double tau, double df, const Plan& p) {
  int cell;
  double frac;
  grid_coord32(t, tau, df, (double)p.n, (int)p.n, cell, frac);
  return cell >> p.Tb_shift;
}

// Sorted fast path: the bins of consecutive points are non-decreasing, so the
// bin starts are the positions where the bin index steps up.  A descent sets
// need_sort and the counting sort below rebuilds everything.
__global__ __launch_bounds__(kThreads) void k_bins_sorted(CallArgs a, Plan p, Work w) {
  const DevStats* st = w.stats;
  if (st->status != 0 || st->need_sort) return;
  const double tau = st->tau;
  const int64_t nd = a.nd;
  const int64_t nb = p.nbins;
  const int kfirst = point_bin(a.t[0], tau, a.df, p);
  const int klast = point_bin(a.t[nd - 1], tau, a.df, p);
  const int64_t total = nd > nb + 1 ? nd : nb + 1;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads) {
    if (i <= nb) {
      if (i <= kfirst) w.bin_start[i] = 0;
      else if (i > klast) w.bin_start[i] = (int)nd;
    }
    if (i >= 1 && i < nd) {
      const int kp = point_bin(a.t[i - 1], tau, a.df, p);
      const int kc = point_bin(a.t[i], tau, a.df, p);
      if (kc < kp) {
        atomicOr(&w.stats->need_sort, 1);
      } else {
        for (int b = kp + 1; b <= kc; ++b) w.bin_start[b] = (int)i;
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_sort_fill(Plan p, Work w) {
  const DevStats* st = w.stats;
  if (st->status != 0 || !st->need_sort) return;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i <= p.nbins;
       i += (int64_t)gridDim.x * kThreads)
    w.bin_count[i] = 0;
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
constexpr int kScanChunk = 2048;  // 256 threads x 8

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

__global__ __launch_bounds__(kThreads) void k_scan2(int64_t nchunks, Work w) {
  const DevStats* st = w.stats;
  if (st->status != 0 || !st->need_sort) return;
  __shared__ int s[kThreads];
  int carry = 0;
  for (int64_t base = 0; base < nchunks; base += kThreads) {
    int64_t i = base + threadIdx.x;
    int v = i < nchunks ? w.scan_part[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
      int x = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += x;
      __syncthreads();
    }
    if (i < nchunks) w.scan_part[i] = carry + s[threadIdx.x] - v;
    int tot = s[kThreads - 1];
    __syncthreads();
    carry += tot;
  }
}

__global__ __launch_bounds__(kThreads) void k_scan3(Plan p, Work w) {
  const DevStats* st = w.stats;
  if (st->status != 0 || !st->need_sort) return;
  const int64_t cnt = p.nbins + 1;
  const int add = w.scan_part[blockIdx.x];
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
    w.ts[pos] = t;
    if (a.periodogram) {
      w.ys[pos] = a.y[j];
      w.dys[pos] = a.dy ? a.dy[j] : 1.0;
    } else {
      w.hs[pos] = a.h[j];
    }
  }
}

// ============================================================================
// Spreading.  One workgroup per tile of T consecutive cells of one row of the
// [nrows][S1] view of the grid.  It gathers every point whose kernel support
// (w cells around u) meets the tile, accumulates the kernel-weighted
// strengths in LDS and writes the tile once: no global atomics, no halo
// exchange, and the result does not depend on how tiles are scheduled.
// Rows that no kernel support reaches are not written; their flag tells the
// first FFT pass to treat them as zero.
// ============================================================================
__device__ __forceinline__ int64_t floordiv2(int64_t x) { return x >= 0 ? x / 2 : -((-x + 1) / 2); }
__device__ __forceinline__ int64_t ceildiv2(int64_t x) { return x >= 0 ? (x + 1) / 2 : -((-x) / 2); }

// Append the point ranges of the cyclic cell interval [c0, c1) (of the
// binning geometry) to rb/re (LDS arrays), at most two ranges.
__device__ __forceinline__ void add_cell_range(int* rb, int* re, int& cnt, int64_t c0, int64_t c1,
                                               const Plan& p, const int* bs, int nd) {
  const int64_t n = p.n;
  if (c1 - c0 >= n) {
    rb[cnt] = 0;
    re[cnt] = nd;
    ++cnt;
    return;
  }
  int64_t x0 = c0 % n;
  if (x0 < 0) x0 += n;
  const int64_t x1 = x0 + (c1 - c0);
  const int64_t e1 = x1 <= n ? x1 : n;
  rb[cnt] = bs[x0 >> p.Tb_shift];
  re[cnt] = bs[((e1 - 1) >> p.Tb_shift) + 1];
  ++cnt;
  if (x1 > n) {
    rb[cnt] = bs[0];
    re[cnt] = bs[((x1 - n - 1) >> p.Tb_shift) + 1];
    ++cnt;
  }
}

// Points whose geometry-GEO coordinate may fall in the cyclic interval
// [c0, c1); returns the number of ranges written (<= 4).
template <int GEO>
__device__ __forceinline__ int gather_ranges(int* rb, int* re, int64_t c0, int64_t c1,
                                             const Plan& p, const int* bs, int nd) {
  int cnt = 0;
  if (GEO == 1) {
    add_cell_range(rb, re, cnt, c0, c1, p, bs, nd);
  } else {
    // u_2f = 2 u_f mod n: the cyclic interval [c0, c1) has the two pre-images
    // [c0/2, c1/2) and [(c0+n)/2, (c1+n)/2) in u_f (one cell of slack each side).
    if (c1 - c0 + 8 >= p.n) {
      rb[0] = 0;
      re[0] = nd;
      return 1;
    }
    add_cell_range(rb, re, cnt, floordiv2(c0) - 1, ceildiv2(c1) + 1, p, bs, nd);
    add_cell_range(rb, re, cnt, floordiv2(c0 + p.n) - 1, ceildiv2(c1 + p.n) + 1, p, bs, nd);
  }
  return cnt;
}

template <typename Real, int GEO, int NG>
__global__ __launch_bounds__(kThreads) void k_spread(CallArgs a, Plan p, Work w, int gbase,
                                                     unsigned char* rowflag) {
  using T2 = typename cplx<Real>::T;
  __shared__ Real acc[NG][2][kTileMax];
  __shared__ int rb[8], re[8];
  __shared__ int snr, sactive;
  const DevStats* stp = w.stats;
  if (stp->status != 0) return;
  const int tid = threadIdx.x;
  const int tiles_per_row = (int)(p.S1 / p.T);
  const int ntiles = tiles_per_row * (int)p.nrows;
  const int tile = (int)xcd_remap(blockIdx.x, ntiles);
  const int row = tile / tiles_per_row;
  const int seg = tile - row * tiles_per_row;
  const int64_t a0 = (int64_t)row * p.S1 + (int64_t)seg * p.T;
  const int h = (int)ceil(p.hw) + 1;
  const int nd = (int)a.nd;
  const int* bs = w.bin_start;

  if (tid == 0) {
    int cnt = gather_ranges<GEO>(rb, re, (int64_t)row * p.S1 - h, (int64_t)(row + 1) * p.S1 + h,
                                 p, bs, nd);
    int tot = 0;
    for (int i = 0; i < cnt; ++i) tot += re[i] - rb[i];
    const int active = tot > 0;
    if (seg == 0) rowflag[row] = (unsigned char)active;
    sactive = active;
    snr = active ? gather_ranges<GEO>(rb, re, a0 - h, a0 + p.T + h, p, bs, nd) : 0;
  }
  __syncthreads();
  if (!sactive) return;
  const int T = p.T;
  for (int x = tid; x < T; x += kThreads) {
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      acc[g][0][x] = 0;
      acc[g][1][x] = 0;
    }
  }
  __syncthreads();

  const bool sorted = !stp->need_sort;
  const double tau = stp->tau;
  const double invW = 1.0 / stp->W;
  const double ysub = stp->ysub;
  const double gstep = GEO * a.df;
  const int n = (int)p.n;
  const double nreal = (double)p.n;
  const int wd = p.w;
  const double hw = p.hw;
  const double inv_hw = 1.0 / p.hw;
  const Real beta = (Real)p.beta;
  // a kernel support can meet the tile at most once unless the tile spans
  // nearly the whole periodic grid
  const bool wrap_free = T <= n - wd;
  const double* tt = sorted ? a.t : w.ts;
  const double* yy = a.periodogram ? (sorted ? a.y : w.ys) : (sorted ? a.h : w.hs);
  const double* dd = sorted ? a.dy : w.dys;
  const bool have_dy = a.periodogram && (sorted ? a.dy != nullptr : true);
  const int nr = snr;
  for (int r = 0; r < nr; ++r) {
    const int jend = re[r];
    for (int j = rb[r] + tid; j < jend; j += kThreads) {
      const double t = tt[j];
      int cell;
      double frac;
      grid_coord32(t, tau, gstep, nreal, n, cell, frac);
      const int o0 = (int)ceil(frac - hw);
      int lb = cell + o0 - (int)a0;  // in (-2n, n)
      if (lb < 0) lb += n;
      if (lb < 0) lb += n;
      if (lb > n - wd) lb -= n;
      if (wrap_free && (lb >= T || lb + wd <= 0)) continue;
      double pc, ps;
      prephase(t, tau, a.fch, a.fcl, pc, ps);
      Real hre[NG], him[NG];
      if (a.periodogram) {
        double wj = 1.0;
        if (have_dy) {
          const double dv = dd[j];
          wj = 1.0 / (dv * dv);
        }
        const double wh = wj * invW;
        if (GEO == 1) {
          const double yt = yy[j] - ysub;
          hre[0] = (Real)(wh * yt * pc);
          him[0] = (Real)(wh * yt * ps);
          if (NG > 1) {
            hre[NG - 1] = (Real)(wh * pc);
            him[NG - 1] = (Real)(wh * ps);
          }
        } else {
          // exp(2 i theta) from exp(i theta)
          hre[0] = (Real)(wh * (pc * pc - ps * ps));
          him[0] = (Real)(wh * (2.0 * pc * ps));
        }
      } else {
        const double hv = yy[j];
        hre[0] = (Real)(hv * pc);
        him[0] = (Real)(hv * ps);
      }
      for (int k = 0; k < wd; ++k) {
        int loc = lb + k;
        if (loc < 0) loc += n;
        else if (loc >= n) loc -= n;
        if (loc >= T) continue;
        const Real z = (Real)(((double)(o0 + k) - frac) * inv_hw);
        const Real v = es_kernel(z, beta);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          atomicAdd(&acc[g][0][loc], v * hre[g]);
          atomicAdd(&acc[g][1][loc], v * him[g]);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    T2* out = reinterpret_cast<T2*>(w.grid[gbase + g]);
    for (int x = tid; x < T; x += kThreads) {
      T2 v;
      v.x = acc[g][0][x];
      v.y = acc[g][1][x];
      out[a0 + x] = v;
    }
  }
}

// ============================================================================
// FFT passes.
// ============================================================================
template <typename Real>
struct PassBufs {
  typename cplx<Real>::T* in[3];
  typename cplx<Real>::T* out[3];
  const unsigned char* rowflag[3];
};

// A first/middle pass: workgroup = C consecutive columns s of one outer index
// p; loads L x C elements (C contiguous per row, 128-256 B segments),
// transforms along L in LDS, applies the inter-pass twiddle and stores with
// the outer index and k transposed.  Dynamic LDS: L*C elements + L twiddles
// + L row flags.
template <typename Real, int EMAX, int NT>
__global__ __launch_bounds__(NT) void k_fft_pass(PassBufs<Real> b, FftPass ps,
                                                 const typename cplx<Real>::T* tw,
                                                 const DevStats* st) {
  using T2 = typename cplx<Real>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  if (st->status != 0) return;
  const int g = blockIdx.y;
  const int tid = threadIdx.x;
  const int L = ps.L, C = ps.C, csh = ps.cshift;
  T2* buf = reinterpret_cast<T2*>(smem);
  T2* twL = buf + L * C;
  unsigned char* rf = reinterpret_cast<unsigned char*>(twL + L);
  const int64_t S = ps.S, P = ps.P;
  const int64_t nsb = (S + C - 1) / C;
  const int64_t blk = xcd_remap(blockIdx.x, (int64_t)gridDim.x);
  const int64_t pidx = blk / nsb;
  const int64_t s0 = (blk - pidx * nsb) * C;
  const int ceff = (int)((S - s0) < C ? (S - s0) : C);
  const T2* in = b.in[g];
  T2* out = b.out[g];
  const unsigned char* rflag = b.rowflag[g];
  for (int x = tid; x < L; x += NT) {
    twL[x] = tw[ps.twL_off + x];
    rf[x] = rflag ? rflag[x] : (unsigned char)1;
  }
  __syncthreads();
  const int E = L * C;
  const int64_t inbase = pidx * (int64_t)L * S + s0;
  constexpr int PER = (EMAX + NT - 1) / NT;
  T2 v[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + i * NT;
    v[i] = czero<T2>();
    if (e < E) {
      const int l = e >> csh;
      const int c = e & (C - 1);
      if (c < ceff && rf[l]) v[i] = in[inbase + (int64_t)l * S + c];
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + i * NT;
    if (e < E) buf[e] = v[i];
  }
  __syncthreads();
  lds_fft<EMAX, NT>(buf, L, C, 1, C, ps.rad, ps.nrad, twL, false);
  const int64_t mask = ((int64_t)1 << ps.bshift) - 1;
  const T2* tlo = tw + ps.twlo_off;
  const T2* thi = tw + ps.twhi_off;
  const int64_t PS = P * S;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + i * NT;
    if (e < E) {
      const int k = e >> csh;
      const int c = e & (C - 1);
      if (c < ceff) {
        const int64_t s = s0 + c;
        T2 x = buf[e];
        const int64_t q = s * k;
        if (q) x = cmul(x, cmul(thi[q >> ps.bshift], tlo[q & mask]));
        out[(int64_t)k * PS + pidx * S + s] = x;
      }
    }
  }
}

// Power of the floating-mean Lomb-Scargle fit from the three normalised sums
// A = sum w^ y~ e^{iwt}, B = sum w^ e^{iwt}, B2 = sum w^ e^{2iwt}
// (w^ = w / W).  cos^2 and sin^2 sums follow from B2 by the double-angle
// identities; the 2x2 fit is solved in closed form (tau-free form).
__device__ __forceinline__ double ls_power(double Ar, double Ai, double Br, double Bi, double B2r,
                                           double B2i, const DevStats& st, int norm,
                                           int fit_mean) {
  double CC = 0.5 * (1.0 + B2r);
  double SS = 0.5 * (1.0 - B2r);
  double CS = 0.5 * B2i;
  double YC = Ar, YS = Ai;
  if (fit_mean) {
    CC -= Br * Br;
    SS -= Bi * Bi;
    CS -= Br * Bi;
    YC -= st.Ybar * Br;
    YS -= st.Ybar * Bi;
  }
  const double D = CC * SS - CS * CS;
  if (!(D > 0.0)) return 0.0;
  const double N = SS * YC * YC + CC * YS * YS - 2.0 * CS * YC * YS;
  const double YYD = st.YY * D;
  switch (norm) {
    case 1:
      return N / (YYD - N);
    case 2:
      return -log1p(-N / YYD);
    case 3:
      return 0.5 * st.W * N / D;
    default:
      return N / YYD;
  }
}

// Last pass: D rows of length L per workgroup for the G grids, transformed in
// LDS; output k of row p is the mode m = p + P k.  Deconvolution, crop to the
// nf requested modes and (G = 3) the power are fused into the store.
// Dynamic LDS: G*D*(L+1) elements + L twiddles.
template <typename Real, int G, int EMAX, int NT>
__global__ __launch_bounds__(NT) void k_fft_last(PassBufs<Real> b, FftPass ps, Plan pl,
                                                 CallArgs a, const typename cplx<Real>::T* tw,
                                                 const double* inv_phihat, const DevStats* stp) {
  using T2 = typename cplx<Real>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  if (stp->status != 0) return;
  const int tid = threadIdx.x;
  const int L = ps.L, D = ps.C;
  const int Lp = L + 1;
  T2* buf = reinterpret_cast<T2*>(smem);
  T2* twL = buf + G * D * Lp;
  const int64_t P = ps.P;
  const int64_t nblk = (P + D - 1) / D;
  const int64_t blk = xcd_remap(blockIdx.x, nblk);
  const int64_t p0 = blk * D;
  const int deff = (int)((P - p0) < D ? (P - p0) : D);
  for (int x = tid; x < L; x += NT) twL[x] = tw[ps.twL_off + x];
  const int E = D * L;
  constexpr int PER = (EMAX / G + NT - 1) / NT;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const T2* in = b.in[g] + p0 * (int64_t)L;
    T2 v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      v[i] = czero<T2>();
      if (e < E && e < deff * L) v[i] = in[e];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      if (e < E) {
        const int d = e / L;
        const int l = e - d * L;
        buf[(g * D + d) * Lp + l] = v[i];
      }
    }
  }
  __syncthreads();
  lds_fft<EMAX, NT>(buf, L, G * D, Lp, 1, ps.rad, ps.nrad, twL, true);
  const DevStats st = *stp;
  const int64_t n = pl.n, nf = pl.nf, K = pl.K;
  for (int e = tid; e < E; e += NT) {
    const int d = e % D;
    const int k = e / D;
    if (d >= deff) continue;
    const int64_t m = p0 + d + P * (int64_t)k;
    const int64_t mm = (m <= nf - 1 - K) ? m : m - n;
    const int64_t kout = mm + K;
    if (kout < 0 || kout >= nf) continue;
    const double ip = inv_phihat[mm < 0 ? -mm : mm];
    if (G == 3) {
      const T2 A = buf[(0 * D + d) * Lp + k];
      const T2 B = buf[(1 * D + d) * Lp + k];
      const T2 B2 = buf[(2 * D + d) * Lp + k];
      double pw = ls_power((double)A.x * ip, (double)A.y * ip, (double)B.x * ip, (double)B.y * ip,
                           (double)B2.x * ip, (double)B2.y * ip, st, a.norm, a.fit_mean);
      if (kout == a.kzero) pw = 0.0;
      a.power[kout] = pw;
    } else {
      const T2 A = buf[d * Lp + k];
      double2 v = make_double2((double)A.x * ip, (double)A.y * ip);
      reinterpret_cast<double2*>(a.sums)[kout] = v;
    }
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

// ============================================================================
// Host launchers
// ============================================================================
static inline unsigned grid_for(int64_t work, int64_t cap) {
  int64_t b = (work + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

hipError_t launch_phihat(double* inv_phihat, int64_t K, double w, double n, const double* z,
                         const double* gphi, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_phihat, dim3(grid_for(K + 1, 1 << 30)), dim3(kThreads), 0, s, inv_phihat,
                     K, w, n, z, gphi, q);
  return hipGetLastError();
}

template <typename Real>
static hipError_t launch_path_t(const CallArgs& a, const Plan& p, const Work& w, hipStream_t s,
                                const StageHook* hook) {
  using T2 = typename cplx<Real>::T;
  constexpr bool f64 = sizeof(Real) == 8;
  constexpr int EMID = f64 ? kEmid64 : kEmid32;
  constexpr int ELAST = f64 ? kElast64 : kElast32;
  const int G = a.periodogram ? 3 : 1;
  auto mark = [&](int stage, int begin) {
    if (hook) hook->fn(hook->ud, stage, begin, s);
  };
  mark(kStageStats, 1);
  hipLaunchKernelGGL(k_stats, dim3(kStatsBlocks), dim3(kThreads), 0, s, a, w);
  mark(kStageStats, 0);
  mark(kStageBin, 1);
  const int64_t nbt = (a.nd > p.nbins + 1 ? a.nd : p.nbins + 1);
  hipLaunchKernelGGL(k_bins_sorted, dim3(grid_for(nbt, 1 << 20)), dim3(kThreads), 0, s, a, p, w);
  // counting-sort path: these exit at once unless a descent was found
  const unsigned sort_blocks = grid_for(a.nd > p.nbins ? a.nd : p.nbins, 512);
  hipLaunchKernelGGL(k_sort_fill, dim3(sort_blocks), dim3(kThreads), 0, s, p, w);
  hipLaunchKernelGGL(k_sort_hist, dim3(sort_blocks), dim3(kThreads), 0, s, a, p, w);
  const int64_t nchunks = (p.nbins + 1 + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan1, dim3((unsigned)nchunks), dim3(kThreads), 0, s, p, w);
  hipLaunchKernelGGL(k_scan2, dim3(1), dim3(kThreads), 0, s, nchunks, w);
  hipLaunchKernelGGL(k_scan3, dim3((unsigned)nchunks), dim3(kThreads), 0, s, p, w);
  hipLaunchKernelGGL(k_sort_scatter, dim3(sort_blocks), dim3(kThreads), 0, s, a, p, w);
  mark(kStageBin, 0);

  const int64_t ntiles = (p.S1 / p.T) * p.nrows;
  if (a.periodogram) {
    mark(kStageSpreadF, 1);
    hipLaunchKernelGGL((k_spread<Real, 1, 2>), dim3((unsigned)ntiles), dim3(kThreads), 0, s, a, p,
                       w, 0, w.rowflag_f);
    mark(kStageSpreadF, 0);
    mark(kStageSpread2F, 1);
    hipLaunchKernelGGL((k_spread<Real, 2, 1>), dim3((unsigned)ntiles), dim3(kThreads), 0, s, a, p,
                       w, 2, w.rowflag_2f);
    mark(kStageSpread2F, 0);
  } else {
    mark(kStageSpreadF, 1);
    hipLaunchKernelGGL((k_spread<Real, 1, 1>), dim3((unsigned)ntiles), dim3(kThreads), 0, s, a, p,
                       w, 0, w.rowflag_f);
    mark(kStageSpreadF, 0);
  }
  const T2* tw = reinterpret_cast<const T2*>(w.tw);
  // passes 0 .. npass-2
  T2* cur[3];
  T2* alt[3];
  for (int g = 0; g < 3; ++g) {
    cur[g] = reinterpret_cast<T2*>(w.grid[g]);
    alt[g] = reinterpret_cast<T2*>(w.grid2[g]);
  }
  for (int ip = 0; ip + 1 < p.npass; ++ip) {
    const FftPass& ps = p.pass[ip];
    PassBufs<Real> b;
    for (int g = 0; g < 3; ++g) {
      b.in[g] = cur[g];
      b.out[g] = (ip == 0) ? cur[g] : alt[g];
      b.rowflag[g] = (ip == 0) ? (g == 2 ? w.rowflag_2f : w.rowflag_f) : nullptr;
    }
    const int64_t nblk = ps.P * ((ps.S + ps.C - 1) / ps.C);
    const size_t lds = sizeof(T2) * (size_t)(ps.L * ps.C + ps.L) + (size_t)ps.L + 16;
    mark(kStagePass0 + ip, 1);
    hipLaunchKernelGGL((k_fft_pass<Real, EMID, kThreads>), dim3((unsigned)nblk, G),
                       dim3(kThreads), lds, s, b, ps, tw, w.stats);
    mark(kStagePass0 + ip, 0);
    if (ip > 0) {
      for (int g = 0; g < 3; ++g) {
        T2* tmp = cur[g];
        cur[g] = alt[g];
        alt[g] = tmp;
      }
    }
  }
  {
    const FftPass& ps = p.pass[p.npass - 1];
    PassBufs<Real> b;
    for (int g = 0; g < 3; ++g) {
      b.in[g] = cur[g];
      b.out[g] = nullptr;
      b.rowflag[g] = nullptr;
    }
    const int64_t nblk = (ps.P + ps.C - 1) / ps.C;
    const size_t lds = sizeof(T2) * (size_t)(G * ps.C * (ps.L + 1) + ps.L);
    mark(kStageLast, 1);
    if (a.periodogram)
      hipLaunchKernelGGL((k_fft_last<Real, 3, ELAST, kThreadsLast>), dim3((unsigned)nblk),
                         dim3(kThreadsLast), lds, s, b, ps, p, a, tw, w.inv_phihat, w.stats);
    else
      hipLaunchKernelGGL((k_fft_last<Real, 1, ELAST, kThreadsLast>), dim3((unsigned)nblk),
                         dim3(kThreadsLast), lds, s, b, ps, p, a, tw, w.inv_phihat, w.stats);
    mark(kStageLast, 0);
  }
  return hipGetLastError();
}

hipError_t launch_path(const CallArgs& a, const Plan& p, const Work& w, hipStream_t s,
                       const StageHook* hook) {
  if (p.prec == 1) return launch_path_t<float>(a, p, w, s, hook);
  return launch_path_t<double>(a, p, w, s, hook);
}

}  // namespace mils
