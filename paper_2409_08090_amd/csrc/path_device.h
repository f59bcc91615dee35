// path_device.h -- device-side building blocks of the NUFFT Lomb-Scargle
// path, shared by the single-series kernels (kernels.hip) and the persistent
// batched kernel (batch.hip): moment merging, point binning, tile spreading,
// one workgroup's share of an FFT pass, and the power assembly.
#pragma once

#include <hip/hip_runtime.h>

#include "device_math.h"
#include "fft_core.h"
#include "mils_internal.h"

namespace mils {

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


__device__ __forceinline__ int point_bin(double t, double tau, double df, const Plan& p) {
  int cell;
  double frac;
  grid_coord32(t, tau, df, (double)p.n, (int)p.n, cell, frac);
  return cell >> p.Tb_shift;
}


constexpr int kScanChunk = 2048;  // 256 threads x 8


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

// The plan's kernel table is read-only for the whole launch: reading it
// through the constant address space lets the compiler use scalar loads (one
// per wave, not per lane) and feed the coefficients to the FMAs from SGPRs.
template <typename Real>
using ConstPtr = const __attribute__((address_space(4))) Real*;

// Whether any kernel support of geometry GEO reaches row r of the
// [nrows][S1] view of the grid (h: half-width in cells, rounded up, plus one).
template <int GEO>
__device__ __forceinline__ bool row_active(int64_t r, int h, const Plan& p, const int* bs, int nd) {
  int rb[4], re[4];
  const int cnt = gather_ranges<GEO>(rb, re, r * p.S1 - h, (r + 1) * p.S1 + h, p, bs, nd);
  int tot = 0;
  for (int i = 0; i < cnt; ++i) tot += re[i] - rb[i];
  return tot > 0;
}

// Per-point records of one chunk of NT points of a spreading tile (LDS): the
// first covered cell relative to the tile (kSpreadNone: the point misses the
// tile), the kernel argument u and the NG complex strengths (component c of
// grid g at h[(2g + c) NT + i]).
constexpr int kSpreadNone = -(1 << 30);
template <typename Real, int NG, int NT>
struct SpreadRecords {
  int lb[NT];
  Real u[NT];
  Real h[2 * NG * NT];
};

// Spread one tile of geometry GEO into NG grids: cells [tile*T, tile*T + T)
// of the flat grid, where T either divides the row length S1 of the
// [nrows][S1] view or is a whole number of rows.  Unless KNOWN (the caller
// already knows that the tile lies in an active row and has written the row
// flags), the flag of every row that starts inside the tile is written and a
// tile of inactive rows returns at once.  acc: LDS accumulator of NG*2*tcap
// doubles (T <= tcap; doubles for FP32 grids too: on gfx950 the LDS atomic
// add of doubles runs at full rate while that of floats waits ~50x longer
// per instruction); rb, re: 8 LDS ints each; sv: 2 LDS ints.  Called by
// every thread of the workgroup (it contains barriers).
template <typename Real, int GEO, int NG, int NT, bool KNOWN = false, bool DET = false>
__device__ void spread_tile(int tile, int Tt, int tcap, const CallArgs& a, const Plan& p,
                            const Work& w, const DevStats& st, int gbase, unsigned char* rowflag,
                            double* acc, int* rb, int* re, int* sv,
                            SpreadRecords<Real, NG, NT>& rec) {
  using T2 = typename cplx<Real>::T;
  const int tid = threadIdx.x;
  const int64_t a0 = (int64_t)tile * Tt;
  const int T = (int)((p.n - a0) < Tt ? (p.n - a0) : Tt);
  const int h = (int)ceil(p.hw) + 1;
  const int nd = (int)a.nd;
  const int* bs = w.bin_start;
  if (KNOWN) {
    if (tid == 0) {
      sv[1] = 1;
      sv[0] = gather_ranges<GEO>(rb, re, a0 - h, a0 + T + h, p, bs, nd);
    }
  } else if (tid == 0) {
    const int64_t r0 = a0 / p.S1, r1 = (a0 + T - 1) / p.S1;
    int any = 0;
    for (int64_t r = r0; r <= r1; ++r) {
      int cnt = gather_ranges<GEO>(rb, re, r * p.S1 - h, (r + 1) * p.S1 + h, p, bs, nd);
      int tot = 0;
      for (int i = 0; i < cnt; ++i) tot += re[i] - rb[i];
      const int active = tot > 0;
      if (r * p.S1 >= a0) rowflag[r] = (unsigned char)active;
      any |= active;
    }
    sv[1] = any;
    sv[0] = any ? gather_ranges<GEO>(rb, re, a0 - h, a0 + T + h, p, bs, nd) : 0;
  }
  __syncthreads();
  const int active = sv[1];
  const int nr = sv[0];
  if (!active) {
    __syncthreads();  // sv/rb/re are reused by the next tile
    return;
  }
  for (int x = tid; x < T; x += NT) {
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      acc[(2 * g) * tcap + x] = 0;
      acc[(2 * g + 1) * tcap + x] = 0;
    }
  }
  __syncthreads();

  const bool sorted = !st.need_sort;
  const double tau = st.tau;
  const double invW = 1.0 / st.W;
  const double ysub = st.ysub;
  const double gstep = GEO * a.df;
  const int n = (int)p.n;
  const double nreal = (double)p.n;
  const int wd = p.w;
  const double hw = p.hw;
  // a kernel support can meet the tile at most once unless the tile spans
  // nearly the whole periodic grid
  const bool wrap_free = T <= n - wd;
  const double* tt = sorted ? a.t : w.ts;
  const double* yy = a.periodogram ? (sorted ? a.y : w.ys) : (sorted ? a.h : w.hs);
  const double* dd = sorted ? a.dy : w.dys;
  const bool have_dy = a.periodogram && (sorted ? a.dy != nullptr : true);
  // Lane layout of the accumulation: KL consecutive lanes take one point,
  // lane kk adding the kernel value at the point's cell lb + kk; each lane
  // holds the polynomial of its offset kk in registers.  The Q = 64/KL points
  // a wave takes at once lie a quarter chunk apart in the (sorted) point
  // order, so their runs of cells do not meet.
  constexpr int NC = sizeof(Real) == 8 ? kHornerN64 : kHornerN32;
  const int KL = wd <= 16 ? 16 : 32;
  const int kk = tid & (KL - 1);
  const int grp = tid / KL;          // group of KL lanes
  const int Q = 64 / KL;             // groups per wave
  const int wave = tid >> 6;
  const int q = grp - wave * Q;      // group within the wave
  const int nwave = NT / 64;
  const ConstPtr<Real> hc = (ConstPtr<Real>)(p.hcoef);
  Real cf[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) cf[j] = kk < kHornerK ? hc[j * kHornerK + kk] : (Real)0;
  for (int r = 0; r < nr; ++r) {
    const int jend = re[r];
    for (int base = rb[r]; base < jend; base += NT) {
      // (1) one point per thread: its record
      {
        const int j = base + tid;
        int lbv = kSpreadNone;
        if (j < jend) {
          const double t = tt[j];
          int cell;
          double frac;
          grid_coord32(t, tau, gstep, nreal, n, cell, frac);
          const int o0 = (int)ceil(frac - hw);
          int lb = cell + o0 - (int)a0;  // in (-2n, n)
          if (lb < 0) lb += n;
          if (lb < 0) lb += n;
          if (lb > n - wd) lb -= n;
          if (!(wrap_free && (lb >= T || lb + wd <= 0))) {
            lbv = lb;
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
                const double yt = a.unit_y ? 1.0 : yy[j] - ysub;
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
            // kernel argument: u = 2t - 1, t = o0 + hw - frac in [0, 1)
            rec.u[tid] = (Real)(2.0 * ((double)o0 + hw - frac) - 1.0);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
              rec.h[(2 * g) * NT + tid] = hre[g];
              rec.h[(2 * g + 1) * NT + tid] = him[g];
            }
          }
        }
        rec.lb[tid] = lbv;
      }
      __syncthreads();
      // (2) the chunk's points, KL lanes each
      const int cnt = jend - base < NT ? jend - base : NT;
      if constexpr (DET) {
        // fixed order: each thread owns cells x = tid, tid + NT, ... of the
        // tile and adds the chunk's points to them one after another (no
        // atomics; the point order is the binning's, itself fixed)
        for (int i = 0; i < cnt; ++i) {
          const int lb = rec.lb[i];
          if (lb == kSpreadNone) continue;
          const Real u = rec.u[i];
          for (int x = tid; x < T; x += NT) {
            int off = x - lb;  // cell offset within the point's support, mod n
            if (off < 0) off += n;
            else if (off >= n) off -= n;
            if (off >= wd) continue;
            Real v = hc[off];
            for (int jc = 1; jc < NC; ++jc) v = v * u + hc[jc * kHornerK + off];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
              acc[(2 * g) * tcap + x] += (double)(v * rec.h[(2 * g) * NT + i]);
              acc[(2 * g + 1) * tcap + x] += (double)(v * rec.h[(2 * g + 1) * NT + i]);
            }
          }
        }
      } else
      for (int it = 0; it * Q * nwave < NT; ++it) {
        const int i = q * (NT / Q) + wave + nwave * it;  // point slot
        if (i >= cnt) continue;
        const int lb = rec.lb[i];
        if (lb == kSpreadNone || kk >= wd) continue;
        int loc = lb + kk;
        if (loc < 0) loc += n;
        else if (loc >= n) loc -= n;
        if (loc >= T) continue;
        const Real u = rec.u[i];
        Real v = cf[0];
#pragma unroll
        for (int jc = 1; jc < NC; ++jc) v = v * u + cf[jc];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          atomicAdd(&acc[(2 * g) * tcap + loc], (double)(v * rec.h[(2 * g) * NT + i]));
          atomicAdd(&acc[(2 * g + 1) * tcap + loc], (double)(v * rec.h[(2 * g + 1) * NT + i]));
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    T2* out = reinterpret_cast<T2*>(w.grid[gbase + g]);
    for (int x = tid; x < T; x += NT) {
      T2 v;
      v.x = (Real)acc[(2 * g) * tcap + x];
      v.y = (Real)acc[(2 * g + 1) * tcap + x];
      out[a0 + x] = v;
    }
  }
  __syncthreads();
}


template <typename Real>
struct PassBufs {
  typename cplx<Real>::T* in[3];
  typename cplx<Real>::T* out[3];
  const unsigned char* rowflag[3];
};

// A first/middle pass: workgroup = C consecutive columns s of one outer index
// p; loads L x C elements (C contiguous per row, 128-256 B segments),
// transforms along L in LDS, applies the inter-pass twiddle and stores with
// the outer index and k transposed.  One workgroup's share of the pass is the
// logical block blk.  smem: L*C elements + the twiddle table (L entries, or
// tw2_count(L) for TW2) + L row flags; rflag (NULL: every row) marks the
// input rows that are not all zero.  C is a power of two that divides NT,
// so a thread keeps one column c = tid mod C and visits rows l0, l0 + NT/C,
// ... (l0 = tid / C): its global addresses are a base plus uniform strides.
template <typename Real, int EMAX, int NT, bool TW2 = false>
__device__ void fft_pass_block(int64_t blk, const typename cplx<Real>::T* in,
                               typename cplx<Real>::T* out, const unsigned char* rflag,
                               const FftPass& ps, const typename cplx<Real>::T* tw,
                               unsigned char* smem) {
  using T2 = typename cplx<Real>::T;
  const int tid = threadIdx.x;
  const int L = ps.L, C = ps.C, csh = ps.cshift;
  const int ntw = TW2 ? tw2_count(L) : L;
  T2* buf = reinterpret_cast<T2*>(smem);
  T2* twL = buf + L * C;
  const int64_t S = ps.S, P = ps.P;
  const uint32_t nsb = (uint32_t)((S + C - 1) / C);
  const uint32_t pidx32 = (uint32_t)blk / nsb;
  const int64_t pidx = pidx32;
  const int64_t s0 = (int64_t)((uint32_t)blk - pidx32 * nsb) * C;
  const int ceff = (int)((S - s0) < C ? (S - s0) : C);
  const int c = tid & (C - 1);
  const int l0 = tid >> csh;
  const int LS = NT >> csh;  // rows between a thread's consecutive elements
  const bool cok = c < ceff;
  constexpr int PER = (EMAX + NT - 1) / NT;
  const T2* pin = in + pidx * (int64_t)L * S + s0 + (int64_t)l0 * S + c;
  const int64_t istep = (int64_t)LS * S;
  T2 v[PER];
  if (rflag) {
    // first pass: the row flags (and the twiddle table) into LDS, then the
    // loads of the rows that are not all zero
    unsigned char* rf = reinterpret_cast<unsigned char*>(twL + ntw);
    for (int x = tid; x < ntw; x += NT) twL[x] = tw[ps.twL_off + x];
    for (int x = tid; x < L; x += NT) rf[x] = rflag[x];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int l = l0 + i * LS;
      v[i] = czero<T2>();
      if (l < L && cok && rf[l]) v[i] = pin[i * istep];
    }
  } else {
    // later passes: the tile's loads first, then the twiddle table, whose
    // loads and LDS stores overlap the data's latency
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int l = l0 + i * LS;
      v[i] = czero<T2>();
      if (l < L && cok) v[i] = pin[i * istep];
    }
    for (int x = tid; x < ntw; x += NT) twL[x] = tw[ps.twL_off + x];
  }
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (l0 + i * LS < L) buf[tid + i * NT] = v[i];
  // Inter-pass twiddles exp(2 pi i s k / N), N = L S, of this thread's
  // outputs (column s = s0 + c, rows k = l0 + i LS), fetched before the
  // transform so that their latency overlaps it: the first from the table,
  // the others by repeated multiplication with the step exp(2 pi i s LS / N).
  // Threads without outputs (l0 >= L or c >= ceff) and threads with a single
  // output (LS >= L) take index 0 for what they do not use, so every index is
  // below N.
  const int64_t mask = ((int64_t)1 << ps.bshift) - 1;
  const T2* tlo = tw + ps.twlo_off;
  const T2* thi = tw + ps.twhi_off;
  const int64_t scol = s0 + c;
  const int64_t q0 = (cok && l0 < L) ? scol * (int64_t)l0 : 0;
  const int64_t qs = (cok && LS < L) ? scol * (int64_t)LS : 0;
  const T2 w0 = cmul(thi[q0 >> ps.bshift], tlo[q0 & mask]);
  const T2 ws = cmul(thi[qs >> ps.bshift], tlo[qs & mask]);
  __syncthreads();
  lds_fft<EMAX, NT, TW2>(buf, L, C, C, ps.rad, ps.nrad, twL);
  const int64_t PS = P * S;
  T2* pout = out + (int64_t)l0 * PS + pidx * S + s0 + c;
  const int64_t ostep = (int64_t)LS * PS;
  T2 tk = w0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (l0 + i * LS < L && cok) pout[i * ostep] = cmul(buf[tid + i * NT], tk);
    tk = cmul(tk, ws);
  }
  __syncthreads();
}

// Power of the floating-mean Lomb-Scargle fit from the three normalised sums
// A = sum w^ y~ e^{iwt}, B = sum w^ e^{iwt}, B2 = sum w^ e^{2iwt}
// (w^ = w / W).  cos^2 and sin^2 sums follow from B2 by the double-angle
// identities; the 2x2 fit is solved in closed form (tau-free form).
__device__ __forceinline__ double ls_power(double Ar, double Ai, double Br, double Bi, double B2r,
                                           double B2i, const DevStats& st, int norm,
                                           int fit_mean, double dmin) {
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
  // ill-posed: D below the accuracy of the sums, or below 1e-12 of CC SS
  if (!(D > dmin) || !(D > 1e-12 * CC * SS)) return __builtin_nan("");
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
// One workgroup's share of the last pass: D rows starting at p0 = blk*D.
// The G*D rows are interleaved in LDS, element l of row r at l*R + r with
// R = G*D: every wave access of a stage (and of the power readout) is then a
// run of consecutive elements, which the LDS serves without bank conflicts.
// The global loads take the row index fastest (lanes (l, d), D rows of one
// grid), so that their LDS stores are contiguous runs too while each row is
// still read in contiguous 16-element pieces.  smem: L*R elements + the
// twiddle table (L entries, or tw2_count(L) for TW2).  nf and K are those of
// the series (a batched series may use fewer frequencies than its grid's
// plan).
template <typename Real, int G, int EMAX, int NT, bool TW2 = false, bool SER = false>
__device__ void fft_last_block(int64_t blk, const PassBufs<Real>& b, const FftPass& ps,
                               int64_t n, int64_t nf, int64_t K, const CallArgs& a,
                               const typename cplx<Real>::T* tw, const double* inv_phihat,
                               const DevStats& st, unsigned char* smem,
                               const double* lowfix = nullptr, int lowparts = 1,
                               int* nill = nullptr) {
  using T2 = typename cplx<Real>::T;
  const int tid = threadIdx.x;
  const int L = ps.L, D = ps.C;
  const int R = G * D;
  T2* buf = reinterpret_cast<T2*>(smem);
  T2* twL = buf + L * R;
  const int64_t P = ps.P;
  const int64_t p0 = blk * D;
  const int deff = (int)((P - p0) < D ? (P - p0) : D);
  const int E = D * L;
  const int dsh = __builtin_ctz(D);  // D is a power of two
  constexpr int PER = (EMAX / G + NT - 1) / NT;
  // element e = l D + d of the block's rows (row d, position l)
  const int d0 = tid & (D - 1);
  const int l0 = tid >> dsh;
  const int LS = NT >> dsh;  // NT is a multiple of D
  // the rows' loads first, then the twiddle table (its latency hides behind
  // theirs), then the rows into LDS
  T2 v[G][PER];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const T2* in = b.in[g] + (p0 + d0) * (int64_t)L + l0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      v[g][i] = czero<T2>();
      if (l0 + i * LS < L && d0 < deff) v[g][i] = in[i * LS];
    }
  }
  for (int x = tid; x < (TW2 ? tw2_count(L) : L); x += NT) twL[x] = tw[ps.twL_off + x];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int l = l0 + i * LS;
      if (l < L) buf[__mul24(l, R) + g * D + d0] = v[g][i];
    }
  __syncthreads();
  // kernel-transform factors of this thread's outputs, fetched before the
  // transform so that their latency overlaps it (-1: output cropped)
  constexpr int PO = (EMAX / G + NT - 1) / NT;
  double ipv[PO];
  int64_t kov[PO];
#pragma unroll
  for (int i = 0; i < PO; ++i) {
    const int e = tid + i * NT;
    const int d = e & (D - 1);
    const int k = e >> dsh;
    kov[i] = -1;
    ipv[i] = 0.0;
    if (e < E && d < deff) {
      const int64_t m = p0 + d + P * (int64_t)k;
      const int64_t mm = (m <= nf - 1 - K) ? m : m - n;
      const int64_t kout = mm + K;
      if (kout >= 0 && kout < nf) {
        kov[i] = kout;
        ipv[i] = inv_phihat[mm < 0 ? -mm : mm];
      }
    }
  }
  // statistics of the series of a shared-weights group, once per workgroup
  // (uniform loads; the power stores below cannot then force reloads)
  DevStats ser[SER ? G : 1];
  if constexpr (SER) {
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (g < a.nser) ser[g] = *a.sst[g];
  }
  lds_fft<EMAX, NT, TW2>(buf, L, G * D, R, ps.rad, ps.nrad, twL);
#pragma unroll
  for (int i = 0; i < PO; ++i) {
    const int64_t kout = kov[i];
    if (kout < 0) continue;
    const int e = tid + i * NT;
    const int d = e & (D - 1);
    const int k = e >> dsh;
    const double ip = ipv[i];
    if constexpr (SER) {
      // series sharing their weights: grid g holds series g's A; B and B2
      // were computed once for all
      const double2 B = reinterpret_cast<const double2*>(a.bsum_b)[kout];
      const double2 B2 = reinterpret_cast<const double2*>(a.bsum_b2)[kout];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g >= a.nser) continue;
        const DevStats& sg = ser[g];
        if (sg.status != 0) continue;
        const T2 A = buf[k * R + g * D + d];
        double s6[6] = {(double)A.x * ip, (double)A.y * ip, B.x, B.y, B2.x, B2.y};
        const int64_t q = kout - sg.k_lo;
        const bool low = q >= 0 && q < sg.nlow;
        if (low) {
          const double* lf = a.slow[g];
          for (int j = 0; j < 6; ++j) s6[j] = lf[6 * q + j];
          for (int r = 1; r < lowparts; ++r)
            for (int j = 0; j < 6; ++j) s6[j] += lf[r * 6 * kLowMax + 6 * q + j];
        }
        double pw = ls_power(s6[0], s6[1], s6[2], s6[3], s6[4], s6[5], sg, a.norm, a.fit_mean,
                             low ? 0.0 : a.dmin);
        if (kout == a.kzero) pw = 0.0;
        a.spow[g][kout] = pw;
      }
    } else if (G == 3) {
      const T2 A = buf[k * R + d];
      const T2 B = buf[k * R + D + d];
      const T2 B2 = buf[k * R + 2 * D + d];
      double s6[6] = {(double)A.x * ip,  (double)A.y * ip,  (double)B.x * ip,
                      (double)B.y * ip,  (double)B2.x * ip, (double)B2.y * ip};
      const int64_t q = kout - st.k_lo;
      const bool low = lowfix && q >= 0 && q < st.nlow;
      if (low) {
        for (int j = 0; j < 6; ++j) s6[j] = lowfix[6 * q + j];
        for (int r = 1; r < lowparts; ++r)
          for (int j = 0; j < 6; ++j) s6[j] += lowfix[r * 6 * kLowMax + 6 * q + j];
      }
      double pw = ls_power(s6[0], s6[1], s6[2], s6[3], s6[4], s6[5], st, a.norm, a.fit_mean,
                           low ? 0.0 : a.dmin);
      if (kout == a.kzero) pw = 0.0;
      else if (nill && pw != pw) atomicAdd(nill, 1);
      a.power[kout] = pw;
    } else {
      const T2 A = buf[k * R + d];
      double2 v = make_double2((double)A.x * ip, (double)A.y * ip);
      reinterpret_cast<double2*>(a.sums)[kout] = v;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Direct sums near f = 0.
// ---------------------------------------------------------------------------
// The frequencies k in [k_lo, k_lo + nlow) with |f_k| (tmax - tmin) < 2,
// at most kLowMax of them, the ones closest to f = 0.
__device__ __forceinline__ void low_band(const DevStats& st, double f0, double df, int64_t nf,
                                         int64_t& k_lo, int& nlow) {
  nlow = 0;
  k_lo = 0;
  const double span = st.tmax - st.tmin;
  if (!(span > 0.0)) return;
  const double fl = 2.0 / span;
  double ka = ceil((-fl - f0) / df);
  double kb = floor((fl - f0) / df);
  if (ka < 0.0) ka = 0.0;
  if (kb > (double)(nf - 1)) kb = (double)(nf - 1);
  if (kb < ka) return;
  double lo = ka;
  if (kb - ka + 1.0 > (double)kLowMax) {
    double centre = rint(-f0 / df);
    lo = centre - kLowMax / 2;
    if (lo < ka) lo = ka;
    if (lo > kb - kLowMax + 1) lo = kb - kLowMax + 1;
  }
  k_lo = (int64_t)lo;
  nlow = (int)fmin(kb - lo + 1.0, (double)kLowMax);
}

// This thread's contributions to A, B, B2 at frequencies k_lo + g0 + q,
// q < kLowGroup, summed over points j = j0, j0 + stride, ... < nd.  The phase
// at the first frequency is reduced in double-double; the others follow by
// the exact angle-sum recurrence with the step exp(i 2 pi df t).
template <int GRP>
__device__ __forceinline__ void low_accumulate(const CallArgs& a, const DevStats& st, int64_t k_first,
                                               int ng, int64_t j0, int64_t stride,
                                               double* acc /* 6 * GRP */) {
#pragma unroll
  for (int i = 0; i < 6 * GRP; ++i) acc[i] = 0.0;
  // f_first = f0 + k_first df as a double-double
  double kp, ke;
  dd_two_prod((double)k_first, a.df, kp, ke);
  double fh, fe;
  dd_two_sum(a.f0, kp, fh, fe);
  const double fl = fe + ke;
  const double invW = 1.0 / st.W;
  for (int64_t j = j0; j < a.nd; j += stride) {
    const double t = a.t[j];
    double wj = 1.0;
    if (a.dy) {
      const double dv = a.dy[j];
      wj = 1.0 / (dv * dv);
    }
    const double wh = wj * invW;
    const double wy = wh * (a.y[j] - st.ysub);
    double pc, ps, sc, ss;
    prephase(t, st.tau, fh, fl, pc, ps);
    prephase(t, st.tau, a.df, 0.0, sc, ss);
#pragma unroll
    for (int q = 0; q < GRP; ++q) {
      if (q < ng) {
        const double c2 = pc * pc - ps * ps, s2 = 2.0 * pc * ps;
        acc[6 * q + 0] += wy * pc;
        acc[6 * q + 1] += wy * ps;
        acc[6 * q + 2] += wh * pc;
        acc[6 * q + 3] += wh * ps;
        acc[6 * q + 4] += wh * c2;
        acc[6 * q + 5] += wh * s2;
      }
      const double nc = pc * sc - ps * ss;
      ps = pc * ss + ps * sc;
      pc = nc;
    }
  }
}

// Sum `cnt` doubles of every thread of the workgroup; thread i < cnt gets the
// total of value i.  red: LDS of (NT / 64) * cnt doubles.
template <int NT, int CNT>
__device__ __forceinline__ void block_sum(const double* v, double* red, double* out) {
  constexpr int cnt = CNT;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < cnt; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[wave * cnt + i] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w * cnt + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

}  // namespace mils
