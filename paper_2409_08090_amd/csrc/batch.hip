// batch.hip -- periodograms of many independent series in one persistent
// launch (gfx950).
//
// A fixed number of workgroups (slots, ~2 per CU) each own a private
// workspace; a workgroup takes the next series from an atomic queue (ordered
// by decreasing cost on the host), runs the whole path for it -- statistics,
// binning, both spreads, every FFT pass and the fused deconvolution/power --
// with barriers between phases, and moves on.  No workgroup ever waits for
// another, so the launch always drains.  Series are grouped into grid-size
// classes that share a plan (twiddles, kernel transform).
#include <hip/hip_runtime.h>

#include "batch.h"
#include "device_math.h"
#include "fft_core.h"
#include "mils_internal.h"
#include "path_device.h"

namespace mils {

namespace {

constexpr int NT = kThreads;

// Statistics of one series by one workgroup (see k_stats); writes *st.
__device__ void stats_block(const CallArgs& a, DevStats* st, double* sh /* 5*NT */,
                            int* shi /* 2*NT */) {
  const int tid = threadIdx.x;
  double* sW = sh;
  double* sMu = sh + NT;
  double* sM2 = sh + 2 * NT;
  double* sLo = sh + 3 * NT;
  double* sHi = sh + 4 * NT;
  int* sBad = shi;
  int* sUns = shi + NT;
  Moments m = {0.0, 0.0, 0.0};
  double lo = INFINITY, hi = -INFINITY;
  int bad = 0, uns = 0;
  for (int64_t j = tid; j < a.nd; j += NT) {
    const double t = a.t[j];
    const double y = a.y[j];
    double wj = 1.0;
    if (a.dy) {
      const double d = a.dy[j];
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
  for (int s = NT / 2; s > 0; s >>= 1) {
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
    st->W = sW[0];
    st->mu = sMu[0];
    st->M2 = sM2[0];
    st->tmin = sLo[0];
    st->tmax = sHi[0];
    st->invalid = sBad[0];
    st->unsorted = sUns[0];
    st->need_sort = sUns[0];
    st->tau = sLo[0];
    st->ysub = a.center ? sMu[0] : 0.0;
    st->Ybar = a.center ? 0.0 : sMu[0];
    double YY = sM2[0] / sW[0];
    if (!a.fit_mean && !a.center) YY += sMu[0] * sMu[0];
    st->YY = YY;
    int status = 0;
    if (sBad[0]) status = -1;
    else if (!(YY > 0.0)) status = -2;
    st->status = status;
    st->nlow = 0;
    st->k_lo = 0;
  }
  __threadfence();
  __syncthreads();
}

// Binning of one series by one workgroup: the sorted fast path, and a
// counting sort into the slot's sorted copies when the bins are not
// non-decreasing.  Leaves st->need_sort set when the sort ran.
__device__ void bins_block(const CallArgs& a, const Plan& p, const Work& w, DevStats* st,
                           int* shi /* NT + 2 */) {
  const int tid = threadIdx.x;
  const double tau = st->tau;
  const int nd = (int)a.nd;
  const int nb = (int)p.nbins;
  int* flag = shi + NT;
  if (tid == 0) flag[0] = st->unsorted;
  __syncthreads();
  if (!flag[0]) {
    const int kfirst = point_bin(a.t[0], tau, a.df, p);
    const int klast = point_bin(a.t[nd - 1], tau, a.df, p);
    for (int b = tid; b <= nb; b += NT) {
      if (b <= kfirst) w.bin_start[b] = 0;
      else if (b > klast) w.bin_start[b] = nd;
    }
    int desc = 0;
    for (int i = 1 + tid; i < nd; i += NT) {
      const int kp = point_bin(a.t[i - 1], tau, a.df, p);
      const int kc = point_bin(a.t[i], tau, a.df, p);
      if (kc < kp) desc = 1;
      else
        for (int b = kp + 1; b <= kc; ++b) w.bin_start[b] = i;
    }
    if (desc) atomicOr(&flag[0], 1);
  }
  __threadfence();
  __syncthreads();
  if (!flag[0]) return;
  // counting sort
  for (int b = tid; b <= nb; b += NT) w.bin_count[b] = 0;
  __threadfence();
  __syncthreads();
  for (int j = tid; j < nd; j += NT) atomicAdd(&w.bin_count[point_bin(a.t[j], tau, a.df, p)], 1);
  __threadfence();
  __syncthreads();
  // exclusive scan of bin_count[0..nb] in chunks of NT
  int carry = 0;
  for (int base = 0; base <= nb; base += NT) {
    const int i = base + tid;
    const int v = i <= nb ? w.bin_count[i] : 0;
    shi[tid] = v;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
      const int x = tid >= off ? shi[tid - off] : 0;
      __syncthreads();
      shi[tid] += x;
      __syncthreads();
    }
    if (i <= nb) {
      const int ex = carry + shi[tid] - v;
      w.bin_start[i] = ex;
      if (i < nb) w.bin_cursor[i] = ex;
    }
    carry += shi[NT - 1];
    __syncthreads();
  }
  __threadfence();
  __syncthreads();
  for (int j = tid; j < nd; j += NT) {
    const double t = a.t[j];
    const int pos = atomicAdd(&w.bin_cursor[point_bin(t, tau, a.df, p)], 1);
    if (pos < 0 || pos >= nd) continue;  // cannot happen with a consistent histogram
    w.ts[pos] = t;
    w.ys[pos] = a.y[j];
    w.dys[pos] = a.dy ? a.dy[j] : 1.0;
  }
  if (tid == 0) st->need_sort = 1;
  __threadfence();
  __syncthreads();
}

__device__ __noinline__ void batch_stats(const CallArgs& a, DevStats* st, double* sh, int* shi) {
  stats_block(a, st, sh, shi);
}
__device__ __noinline__ void batch_bins(const CallArgs& a, const Plan& p, const Work& w,
                                        DevStats* st, int* shi) {
  bins_block(a, p, w, st, shi);
}

// Direct FP64 sums near f = 0 for one series (see k_lowfreq): lowfix gets
// kLowMax x 6 values, st->k_lo / st->nlow the frequencies they belong to.
__device__ __noinline__ void batch_lowfreq(const CallArgs& a, DevStats* st, double* lowfix,
                                           double* red) {
  const DevStats& s = *st;
  int64_t k_lo;
  int nlow;
  low_band(s, a.f0, a.df, a.nf, k_lo, nlow);
  double acc[6 * kLowGroup];
  for (int g0 = 0; g0 < nlow; g0 += kLowGroup) {
    const int ng = nlow - g0 < kLowGroup ? nlow - g0 : kLowGroup;
    low_accumulate<kLowGroup>(a, s, k_lo + g0, ng, threadIdx.x, NT, acc);
    block_sum<NT, 6 * kLowGroup>(acc, red, lowfix + 6 * g0);
  }
  if (threadIdx.x == 0) {
    st->k_lo = k_lo;
    st->nlow = nlow;
  }
  __threadfence();
  __syncthreads();
}

__device__ __forceinline__ void block_fence() {
  __threadfence();
  __syncthreads();
}

// Phase wrappers kept out of line: each phase gets its own register
// allocation instead of the union of all of them.
// A batched series spreads tiles of several whole rows, up to what the
// dynamic LDS holds for geometry f (two grids), to amortise the per-tile cost.
template <typename Real>
__device__ __forceinline__ int batch_tile_cells() {
  return kBatchLds / (2 * 2 * (int)sizeof(Real));
}
template <typename Real>
__device__ __forceinline__ int batch_tile(const Plan& p) {
  const int cap = batch_tile_cells<Real>();
  return p.S1 <= cap ? (int)(p.S1 * (cap / p.S1)) : p.T;
}
template <typename Real>
__device__ __noinline__ void batch_spread_f(int tile, int Tt, const CallArgs& a, const Plan& p,
                                            const Work& w, const DevStats& st,
                                            unsigned char* smem, int* rb, int* re, int* sv) {
  spread_tile<Real, 1, 2, NT>(tile, Tt, batch_tile_cells<Real>(), a, p, w, st, 0, w.rowflag_f,
                              reinterpret_cast<Real*>(smem), rb, re, sv);
}
template <typename Real>
__device__ __noinline__ void batch_spread_2f(int tile, int Tt, const CallArgs& a, const Plan& p,
                                             const Work& w, const DevStats& st,
                                             unsigned char* smem, int* rb, int* re, int* sv) {
  spread_tile<Real, 2, 1, NT>(tile, Tt, batch_tile_cells<Real>(), a, p, w, st, 2, w.rowflag_2f,
                              reinterpret_cast<Real*>(smem), rb, re, sv);
}
template <typename Real>
__device__ __forceinline__ void batch_pass(int64_t blk, const typename cplx<Real>::T* in,
                                        typename cplx<Real>::T* out, const unsigned char* rf,
                                        const FftPass& ps, const typename cplx<Real>::T* tw,
                                        unsigned char* smem) {
  constexpr int EMID = sizeof(Real) == 8 ? kEmid64 : kEmid32;
  fft_pass_block<Real, EMID, NT>(blk, in, out, rf, ps, tw, smem);
}
template <typename Real>
__device__ __forceinline__ void batch_last(int64_t blk, void* const* grids, const FftPass& ps,
                                        int64_t n, int64_t nf, int64_t K, const CallArgs& a,
                                        const typename cplx<Real>::T* tw, const double* iph,
                                        const DevStats& st, unsigned char* smem,
                                        const double* lowfix) {
  using T2 = typename cplx<Real>::T;
  constexpr int ELAST = sizeof(Real) == 8 ? kElastBatch64 : kElastBatch32;
  PassBufs<Real> b;
  for (int g = 0; g < 3; ++g) {
    b.in[g] = reinterpret_cast<T2*>(grids[g]);
    b.out[g] = nullptr;
    b.rowflag[g] = nullptr;
  }
  fft_last_block<Real, 3, ELAST, NT>(blk, b, ps, n, nf, K, a, tw, iph, st, smem, lowfix);
}

template <typename Real>
__global__ __launch_bounds__(NT, 2) void k_batch(BatchArgs ba) {
  using T2 = typename cplx<Real>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  // per-series state lives in LDS, not in registers, across the phases
  __shared__ Plan sp;
  __shared__ CallArgs sa;
  __shared__ Work sw;
  __shared__ DevStats sst;
  __shared__ BatchCurve sc;
  __shared__ int s_cur;
  __shared__ int rb[8], re[8], sv[2];
  __shared__ int shi[2 * NT + 2];
  __shared__ double slow[6 * kLowMax];
  const int tid = threadIdx.x;
  if (tid == 0) {
    // this slot's workspace
    Work w = ba.w0;
    const size_t off = (size_t)blockIdx.x * ba.slot_stride;
    auto sh = [&](auto* ptr) {
      return ptr ? reinterpret_cast<decltype(ptr)>(reinterpret_cast<char*>(ptr) + off) : ptr;
    };
    w.stats = sh(w.stats);
    w.partials = sh(w.partials);
    w.bin_start = sh(w.bin_start);
    w.bin_count = sh(w.bin_count);
    w.bin_cursor = sh(w.bin_cursor);
    w.scan_part = sh(w.scan_part);
    w.ts = sh(w.ts);
    w.ys = sh(w.ys);
    w.dys = sh(w.dys);
    w.rowflag_f = sh(w.rowflag_f);
    w.rowflag_2f = sh(w.rowflag_2f);
    for (int g = 0; g < 3; ++g) {
      w.grid[g] = sh(reinterpret_cast<char*>(w.grid[g]));
      w.grid2[g] = sh(reinterpret_cast<char*>(w.grid2[g]));
    }
    sw = w;
  }
  for (;;) {
    if (tid == 0) s_cur = (int)atomicAdd(ba.counter, 1u);
    __syncthreads();
    const int ci = s_cur;
    if (ci >= ba.ncurves) break;
    {
      const int* src = reinterpret_cast<const int*>(ba.plans + ba.curves[ci].plan);
      int* dst = reinterpret_cast<int*>(&sp);
      for (int i = tid; i < (int)(sizeof(Plan) / sizeof(int)); i += NT) dst[i] = src[i];
    }
    if (tid == 0) {
      const BatchCurve c = ba.curves[ci];
      sc = c;
      CallArgs a{};
      a.t = ba.t + c.t_off;
      a.y = ba.y + c.t_off;
      a.dy = ba.dy ? ba.dy + c.t_off : nullptr;
      a.nd = c.nd;
      a.nf = c.nf;
      a.f0 = c.f0;
      a.df = c.df;
      a.fch = c.fch;
      a.fcl = c.fcl;
      a.kzero = c.kzero;
      a.norm = ba.norm;
      a.center = ba.center;
      a.fit_mean = ba.fit_mean;
      a.periodogram = 1;
      a.power = ba.power + c.out_off;
      sa = a;
    }
    __syncthreads();
    const Plan& p = sp;
    const CallArgs& a = sa;
    const Work& w = sw;
    batch_stats(a, w.stats, reinterpret_cast<double*>(smem), shi);
    if (w.stats->status != 0) {
      if (tid == 0) ba.status[sc.index] = w.stats->status;
      __syncthreads();
      continue;
    }
    batch_bins(a, p, w, w.stats, shi);
    batch_lowfreq(a, w.stats, slow, reinterpret_cast<double*>(smem));
    if (tid == 0) sst = *w.stats;
    __syncthreads();
    const DevStats& sts = sst;
    const T2* tw = reinterpret_cast<const T2*>(ba.tw[sc.plan]);
    const double* iph = ba.inv_phihat[sc.plan];
    // spreads
    const int Tt = batch_tile<Real>(p);
    const int ntiles = (int)((p.n + Tt - 1) / Tt);
    for (int tile = 0; tile < ntiles; ++tile)
      batch_spread_f<Real>(tile, Tt, a, p, w, sts, smem, rb, re, sv);
    for (int tile = 0; tile < ntiles; ++tile)
      batch_spread_2f<Real>(tile, Tt, a, p, w, sts, smem, rb, re, sv);
    block_fence();
    // FFT passes: pass 0 in place on grid, then grid -> grid2 -> grid ...
    const int npass = p.npass;
    for (int ip = 0; ip + 1 < npass; ++ip) {
      const FftPass& ps = p.pass[ip];
      const int64_t nblk = ps.P * ((ps.S + ps.C - 1) / ps.C);
      for (int g = 0; g < 3; ++g) {
        T2* gr = reinterpret_cast<T2*>(w.grid[g]);
        T2* g2 = reinterpret_cast<T2*>(w.grid2[g]);
        const T2* in = (ip == 0 || ip % 2 == 1) ? gr : g2;
        T2* out = ip == 0 ? gr : (ip % 2 == 1 ? g2 : gr);
        const unsigned char* rf = ip == 0 ? (g == 2 ? w.rowflag_2f : w.rowflag_f) : nullptr;
        for (int64_t blk = 0; blk < nblk; ++blk) batch_pass<Real>(blk, in, out, rf, ps, tw, smem);
      }
      block_fence();
    }
    {
      // the last pass reads grid2 after an odd number of out-of-place passes
      const bool in2 = npass >= 3 && ((npass - 2) % 2 == 1);
      const FftPass& ps = p.pass[npass - 1];
      const int64_t nblk = (ps.P + ps.C - 1) / ps.C;
      for (int64_t blk = 0; blk < nblk; ++blk)
        batch_last<Real>(blk, in2 ? w.grid2 : w.grid, ps, p.n, sc.nf, sc.K, a, tw, iph, sts, smem,
                         slow);
    }
    if (tid == 0) ba.status[sc.index] = 0;
    block_fence();
  }
}

__global__ void k_batch_reset(unsigned int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

}  // namespace

hipError_t launch_batch(const BatchArgs& ba, int nslots, int prec, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, ba.counter);
  if (prec == 1)
    hipLaunchKernelGGL(k_batch<float>, dim3(nslots), dim3(NT), kBatchLds, s, ba);
  else
    hipLaunchKernelGGL(k_batch<double>, dim3(nslots), dim3(NT), kBatchLds, s, ba);
  return hipGetLastError();
}

}  // namespace mils
