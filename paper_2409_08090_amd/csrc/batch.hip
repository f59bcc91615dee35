// batch.hip -- periodograms of many independent series (gfx950).
//
// A batch runs as a short sequence of launches (captured once in a HIP graph
// by the host): one workgroup per series computes its statistics, binning
// and direct low-frequency sums; then each later phase -- both spreads, every
// FFT pass, the last pass with deconvolution and power -- is one launch whose
// workgroups are the tiles of all series of the batch (a host-built work
// list of (series, tile) items), so that every phase has the whole GPU's
// memory parallelism whatever the size mix.  Series are grouped into
// grid-size classes that share a plan (twiddles, kernel transform); each
// series has its own workspace.
#include <hip/hip_runtime.h>

#include <mutex>

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
    st->nill = 0;
    st->nlow = 0;
    st->k_lo = 0;
  }
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
  __syncthreads();
  if (!flag[0]) return;
  // counting sort
  for (int b = tid; b <= nb; b += NT) w.bin_count[b] = 0;
  __syncthreads();
  for (int j = tid; j < nd; j += NT) atomicAdd(&w.bin_count[point_bin(a.t[j], tau, a.df, p)], 1);
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
  __syncthreads();
}

// Direct FP64 sums near f = 0 for one series (see k_lowfreq): lowfix gets
// kLowMax x 6 values, st->k_lo / st->nlow the frequencies they belong to.
__device__ void lowfreq_block(const CallArgs& a, DevStats* st, double* lowfix, double* red) {
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
  __syncthreads();
}

__device__ __forceinline__ CallArgs curve_args(const BatchArgs& ba, const BatchCurve& c) {
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
  a.dmin = ba.dmin;
  a.center = ba.center;
  a.fit_mean = ba.fit_mean;
  a.periodogram = 1;
  a.power = ba.power + c.out_off;
  return a;
}

// Copy of a series' plan into LDS (it is read often and is the same for the
// whole workgroup).
__device__ __forceinline__ void load_plan(const Plan* src, Plan* dst) {
  const int* s = reinterpret_cast<const int*>(src);
  int* d = reinterpret_cast<int*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(Plan) / sizeof(int)); i += blockDim.x) d[i] = s[i];
}

// Per-series prologue: one workgroup per series (series that run in LDS
// return at once).
__global__ __launch_bounds__(NT) void k_bpro(BatchArgs ba) {
  __shared__ double sh[5 * NT];
  __shared__ int shi[2 * NT + 2];
  __shared__ Plan sp;
  const int ci = blockIdx.x;
  if (ba.curves[ci].small) return;
  const BatchCurve c = ba.curves[ci];
  load_plan(ba.plans + c.plan, &sp);
  __syncthreads();
  const CallArgs a = curve_args(ba, c);
  const Work w = ba.works[ci];
  stats_block(a, w.stats, sh, shi);
  if (w.stats->status != 0) {
    if (threadIdx.x == 0) ba.status[c.index] = w.stats->status;
    return;
  }
  bins_block(a, sp, w, w.stats, shi);
  lowfreq_block(a, w.stats, w.lowfix, sh);
  // row flags of both geometries, so that the spread's workgroups of empty
  // rows stop at once
  const int h = (int)ceil(sp.hw) + 1;
  for (int r = threadIdx.x; r < (int)sp.nrows; r += NT) {
    w.rowflag_f[r] = (unsigned char)row_active<1>(r, h, sp, w.bin_start, (int)a.nd);
    w.rowflag_2f[r] = (unsigned char)row_active<2>(r, h, sp, w.bin_start, (int)a.nd);
  }
  if (threadIdx.x == 0) ba.status[c.index] = 0;
}

// Spreading: one workgroup per tile of one series (every tile of every
// series), both geometries (the series' descriptors, flags, statistics and
// plan are fetched once): geometry f into A and B, then geometry 2f into B2,
// each only where the prologue's row flags say a kernel support reaches the
// tile; a tile of empty rows returns after reading its flags.
template <typename Real>
__global__ __launch_bounds__(NT) void k_bspread2(BatchArgs ba, const BatchItem* items) {
  __shared__ double acc[2 * 2 * kTileMax];
  __shared__ int rb[8], re[8], sv[2];
  __shared__ union {
    SpreadRecords<Real, 2, NT> two;
    SpreadRecords<Real, 1, NT> one;
  } rec;
  __shared__ Plan sp;
  const BatchItem it = items[blockIdx.x];
  const BatchCurve c = ba.curves[it.curve];
  const Work& w = ba.works[it.curve];
  const Plan* pl = ba.plans + it.plan;
  // a tile is one row or part of one, or (short rows) several whole rows
  const int64_t a0 = (int64_t)it.sub * pl->T;
  const int64_t r0 = a0 / pl->S1;
  int64_t r1 = (a0 + pl->T - 1) / pl->S1;
  if (r1 >= pl->nrows) r1 = pl->nrows - 1;
  int any_f = 0, any_2f = 0;
  for (int64_t r = r0; r <= r1; ++r) {
    any_f |= w.rowflag_f[r];
    any_2f |= w.rowflag_2f[r];
  }
  if (!any_f && !any_2f) return;
  const DevStats st = *w.stats;
  if (st.status != 0) return;
  load_plan(pl, &sp);
  __syncthreads();
  const CallArgs a = curve_args(ba, c);
  if (any_f)
    spread_tile<Real, 1, 2, NT, true>(it.sub, sp.T, kTileMax, a, sp, w, st, 0, nullptr, acc, rb,
                                      re, sv, rec.two);
  if (any_2f)
    spread_tile<Real, 2, 1, NT, true>(it.sub, sp.T, kTileMax, a, sp, w, st, 2, nullptr, acc, rb,
                                      re, sv, rec.one);
}

// A first/middle FFT pass ip.  FP64: one workgroup per (series, column
// block), which transforms that block of the three grids one after another
// (the series' descriptors and pass parameters are fetched once for the
// three: 10^4-series batch 11.2 -> 9.8 ms).  FP32: one workgroup per (series,
// grid, column block) (three grids per workgroup measured 6.5 -> 7.1 ms).
// Pass 0 works in place on grid; later passes alternate grid -> grid2 ->
// grid.
template <typename Real>
__global__ __launch_bounds__(NT) void k_bpass(BatchArgs ba, const BatchItem* items, int ip) {
  using T2 = typename cplx<Real>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int EMID = sizeof(Real) == 8 ? kEmid64 : kEmid32;
  __shared__ FftPass ps;  // in LDS: its radix list is indexed at run time
  __shared__ int bad;
  const BatchItem it = items[blockIdx.x];
  const Work& w = ba.works[it.curve];  // in place: grid[g] is indexed at run time
  const int cls = it.plan;
  // the pass parameters and the series' status load side by side (both
  // depend on the item only)
  {
    const int* src = reinterpret_cast<const int*>(&ba.plans[cls].pass[ip]);
    int* dst = reinterpret_cast<int*>(&ps);
    for (int i = threadIdx.x; i < (int)(sizeof(FftPass) / sizeof(int)); i += NT) dst[i] = src[i];
    if (threadIdx.x == NT - 1) bad = w.stats->status != 0;
  }
  __syncthreads();
  if (bad) return;
  constexpr int NGW = kBatchPassGrids<Real>;
  const int nblk = (int)(ps.P * ((ps.S + ps.C - 1) / ps.C));
  const int g0 = NGW == 3 ? 0 : it.sub / nblk;
  const int blk = NGW == 3 ? it.sub : it.sub - g0 * nblk;
  const T2* tw = reinterpret_cast<const T2*>(ba.tw[cls]);
  for (int g = g0; g < g0 + NGW; ++g) {
    T2* gr = reinterpret_cast<T2*>(w.grid[g]);
    T2* g2 = reinterpret_cast<T2*>(w.grid2[g]);
    const T2* in = (ip == 0 || ip % 2 == 1) ? gr : g2;
    T2* out = ip == 0 ? gr : (ip % 2 == 1 ? g2 : gr);
    const unsigned char* rf = ip == 0 ? (g == 2 ? w.rowflag_2f : w.rowflag_f) : nullptr;
    fft_pass_block<Real, EMID, NT>(blk, in, out, rf, ps, tw, smem);
    __syncthreads();  // the next grid's tile reuses the LDS
  }
}

// The last pass with deconvolution, crop and power: one workgroup per
// (series, row block).
template <typename Real>
__global__ __launch_bounds__(last_threads<Real>()) void k_blast(BatchArgs ba,
                                                               const BatchItem* items) {
  using T2 = typename cplx<Real>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int ELAST = sizeof(Real) == 8 ? kElast64 : kElast32;
  const BatchItem it = items[blockIdx.x];
  const BatchCurve c = ba.curves[it.curve];
  const Work w = ba.works[it.curve];
  const DevStats st = *w.stats;
  if (st.status != 0) return;
  // no static LDS here: the dynamic part may use all 64 KB
  const Plan* pl = ba.plans + it.plan;
  const int npass = pl->npass;
  const int64_t n = pl->n;
  const FftPass& ps = pl->pass[npass - 1];  // read in place (its radix list is indexed at run time)
  const CallArgs a = curve_args(ba, c);
  const bool in2 = npass >= 3 && ((npass - 2) % 2 == 1);
  PassBufs<Real> b;
  for (int g = 0; g < 3; ++g) {
    b.in[g] = reinterpret_cast<T2*>(in2 ? w.grid2[g] : w.grid[g]);
    b.out[g] = nullptr;
    b.rowflag[g] = nullptr;
  }
  fft_last_block<Real, 3, ELAST, last_threads<Real>()>(it.sub, b, ps, n, c.nf, c.K, a,
                                               reinterpret_cast<const T2*>(ba.tw[it.plan]),
                                               ba.inv_phihat[it.plan], st, smem, w.lowfix, 1);
}

// A series whose three grids fit LDS, whole in one workgroup: statistics and
// direct sums near f = 0 as in the prologue; then each point adds its kernel
// values straight into the LDS grids (FP64 atomics, no binning: any order of
// the additions gives the same sums up to rounding) -- A and B at geometry f,
// B2 at 2f; the three transforms in LDS; deconvolution, crop and power.  The
// grids are FP64 in both precisions (the FP32 form keeps its plan, kernel
// width and polynomial coefficients); nothing but the inputs and the power
// crosses HBM.
template <typename Real>
__global__ __launch_bounds__(NT) void k_bsmall(BatchArgs ba, const BatchItem* items) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sh[5 * NT];
  __shared__ int shi[2 * NT + 2];
  __shared__ Plan sp;
  __shared__ int rad[kSmallMaxRad];
  const int tid = threadIdx.x;
  const int ci = items[blockIdx.x].curve;
  const BatchCurve c = ba.curves[ci];
  load_plan(ba.plans + c.plan, &sp);
  if (tid < c.nsrad) rad[tid] = c.srad[tid];
  __syncthreads();
  const CallArgs a = curve_args(ba, c);
  const Work w = ba.works[ci];
  stats_block(a, w.stats, sh, shi);
  if (w.stats->status != 0) {
    if (tid == 0) ba.status[c.index] = w.stats->status;
    return;
  }
  lowfreq_block(a, w.stats, w.lowfix, sh);
  const DevStats st = *w.stats;
  const int n = (int)sp.n;
  double2* g = reinterpret_cast<double2*>(smem);  // element l of grid q at 3 l + q
  double2* twl = g + 3 * n;
  for (int x = tid; x < 3 * n; x += NT) g[x] = make_double2(0.0, 0.0);
  // two-level table of exp(2 pi i x / n): x < 64, then multiples of 64
  for (int x = tid; x < 64 + (n + 63) / 64; x += NT) {
    const int e = x < 64 ? x : (x - 64) * 64;
    double sv, cv;
    sincospi(2.0 * (double)e / (double)n, &sv, &cv);
    twl[x] = make_double2(cv, sv);
  }
  __syncthreads();
  constexpr int NC = sizeof(Real) == 8 ? kHornerN64 : kHornerN32;
  const ConstPtr<Real> hc = (ConstPtr<Real>)(sp.hcoef);
  const double tau = st.tau, invW = 1.0 / st.W, ysub = st.ysub;
  const double nreal = (double)n, hw = sp.hw;
  const int wd = sp.w;
  for (int64_t j = tid; j < a.nd; j += NT) {
    const double t = a.t[j];
    double wj = 1.0;
    if (a.dy) {
      const double dv = a.dy[j];
      wj = 1.0 / (dv * dv);
    }
    const double wh = wj * invW;
    const double yt = a.y[j] - ysub;
    double pc, ps;
    prephase(t, tau, a.fch, a.fcl, pc, ps);
#pragma unroll
    for (int geo = 1; geo <= 2; ++geo) {
      int cell;
      double frac;
      grid_coord32(t, tau, geo * a.df, nreal, n, cell, frac);
      const int o0 = (int)ceil(frac - hw);
      int lb = cell + o0;  // in (-w, n)
      if (lb < 0) lb += n;
      const Real u = (Real)(2.0 * ((double)o0 + hw - frac) - 1.0);
      const double h0r = geo == 1 ? wh * yt * pc : wh * (pc * pc - ps * ps);
      const double h0i = geo == 1 ? wh * yt * ps : wh * (2.0 * pc * ps);
      const double h1r = wh * pc, h1i = wh * ps;
      for (int kk = 0; kk < wd; ++kk) {
        Real v = hc[kk];
#pragma unroll
        for (int jc = 1; jc < NC; ++jc) v = v * u + hc[jc * kHornerK + kk];
        const double vv = (double)v;
        int loc = lb + kk;
        if (loc >= n) loc -= n;
        if (geo == 1) {
          atomicAdd(&g[3 * loc].x, vv * h0r);
          atomicAdd(&g[3 * loc].y, vv * h0i);
          atomicAdd(&g[3 * loc + 1].x, vv * h1r);
          atomicAdd(&g[3 * loc + 1].y, vv * h1i);
        } else {
          atomicAdd(&g[3 * loc + 2].x, vv * h0r);
          atomicAdd(&g[3 * loc + 2].y, vv * h0i);
        }
      }
    }
  }
  __syncthreads();
  lds_fft<3 * kSmallMaxN, NT, true>(g, n, 3, 3, rad, c.nsrad, twl);
  const int64_t nf = c.nf, K = c.K;
  const double* iph = ba.inv_phihat[c.plan];
  for (int64_t k = tid; k < nf; k += NT) {
    const int64_t mm = k - K;
    const int64_t m = mm < 0 ? mm + n : mm;
    const double ip = iph[mm < 0 ? -mm : mm];
    const double2 A = g[3 * m], B = g[3 * m + 1], B2 = g[3 * m + 2];
    double s6[6] = {A.x * ip, A.y * ip, B.x * ip, B.y * ip, B2.x * ip, B2.y * ip};
    const int64_t q = k - st.k_lo;
    const bool low = q >= 0 && q < st.nlow;
    if (low)
      for (int jj = 0; jj < 6; ++jj) s6[jj] = w.lowfix[6 * q + jj];
    double pw = ls_power(s6[0], s6[1], s6[2], s6[3], s6[4], s6[5], st, a.norm, a.fit_mean,
                         low ? 0.0 : a.dmin);
    if (k == a.kzero) pw = 0.0;
    a.power[k] = pw;
  }
  if (tid == 0) ba.status[c.index] = 0;
}

template <typename Real>
hipError_t launch_t(const BatchLaunch& bl, hipStream_t s) {
  const BatchArgs& ba = bl.args;
  if (bl.nsmall > 0)
    hipLaunchKernelGGL(k_bsmall<Real>, dim3(bl.nsmall), dim3(NT), bl.small_lds, s, ba,
                       bl.small_items);
  hipLaunchKernelGGL(k_bpro, dim3(ba.ncurves), dim3(NT), 0, s, ba);
  if (bl.nspread > 0)
    hipLaunchKernelGGL(k_bspread2<Real>, dim3(bl.nspread), dim3(NT), 0, s, ba, bl.spread_items);
  for (int ip = 0; ip < kMaxPass - 1; ++ip)
    if (bl.npass_items[ip] > 0)
      hipLaunchKernelGGL(k_bpass<Real>, dim3(bl.npass_items[ip]), dim3(NT), bl.pass_lds[ip], s,
                         ba, bl.pass_items[ip], ip);
  if (bl.nlast > 0)
    hipLaunchKernelGGL(k_blast<Real>, dim3(bl.nlast), dim3(last_threads<Real>()), bl.last_lds, s,
                       ba, bl.last_items);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_batch(const BatchLaunch& bl, hipStream_t s) {
  (void)hipGetLastError();  // see launch_path: a handled earlier failure is not this launch's
  return bl.prec == 1 ? launch_t<float>(bl, s) : launch_t<double>(bl, s);
}

hipError_t batch_prepare() {
  // once per device (the serving loop's lanes build batches concurrently;
  // later launches then never meet an attribute change)
  static std::mutex mu;
  static uint64_t done = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  const uint64_t bit = dev < 64 ? (uint64_t)1 << dev : 0;
  if (bit && (done & bit)) return hipSuccess;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bsmall<double>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallLdsCap);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bsmall<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallLdsCap);
  if (e == hipSuccess) done |= bit;
  return e;
}

}  // namespace mils
