// fft_core.h -- LDS-resident mixed-radix Stockham FFT building blocks
// (sign +, unnormalised: X_m = sum_l x_l exp(+2 pi i l m / L)).
//
// A workgroup holds `ncol` independent columns of length L in LDS; element l
// of column c sits at buf[c * cs + l * ls].  Each stage of radix R reads R
// elements at stride L/R, applies the stage twiddles, takes a radix-R DFT in
// registers and writes the outputs to their self-sorted positions (Stockham
// autosort), so no bit reversal is needed.  All reads of a stage complete
// (barrier) before any write, which lets the stage work in place.
#pragma once

#include "device_math.h"
#include "mils_internal.h"

namespace mils {

// ---- radix-R DFTs with the + sign -----------------------------------------
template <typename T2>
__device__ __forceinline__ void dft2(T2* a) {
  T2 t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <typename T2>
__device__ __forceinline__ void dft3(T2* a) {
  using R = decltype(a[0].x);
  const R c = (R)-0.5;
  const R s = (R)0.86602540378443864676372317075294;  // sin(2 pi / 3)
  T2 b = cadd(a[1], a[2]);
  T2 d = csub(a[1], a[2]);
  T2 y0 = cadd(a[0], b);
  T2 m;
  m.x = a[0].x + c * b.x;
  m.y = a[0].y + c * b.y;
  T2 sd = cmuli(cscale(d, s));
  a[0] = y0;
  a[1] = cadd(m, sd);
  a[2] = csub(m, sd);
}

template <typename T2>
__device__ __forceinline__ void dft4(T2* a) {
  T2 s02 = cadd(a[0], a[2]);
  T2 d02 = csub(a[0], a[2]);
  T2 s13 = cadd(a[1], a[3]);
  T2 d13 = cmuli(csub(a[1], a[3]));
  a[0] = cadd(s02, s13);
  a[2] = csub(s02, s13);
  a[1] = cadd(d02, d13);
  a[3] = csub(d02, d13);
}

template <typename T2>
__device__ __forceinline__ void dft5(T2* a) {
  using R = decltype(a[0].x);
  const R c1 = (R)0.30901699437494742410229341718282;   // cos(2 pi / 5)
  const R s1 = (R)0.95105651629515357211643933337938;   // sin(2 pi / 5)
  const R c2 = (R)-0.80901699437494742410229341718282;  // cos(4 pi / 5)
  const R s2 = (R)0.58778525229247312916870595463907;   // sin(4 pi / 5)
  T2 b1 = cadd(a[1], a[4]), d1 = csub(a[1], a[4]);
  T2 b2 = cadd(a[2], a[3]), d2 = csub(a[2], a[3]);
  T2 y0 = cadd(a[0], cadd(b1, b2));
  T2 r1, r2, i1, i2;
  r1.x = a[0].x + c1 * b1.x + c2 * b2.x;
  r1.y = a[0].y + c1 * b1.y + c2 * b2.y;
  r2.x = a[0].x + c2 * b1.x + c1 * b2.x;
  r2.y = a[0].y + c2 * b1.y + c1 * b2.y;
  i1.x = s1 * d1.x + s2 * d2.x;
  i1.y = s1 * d1.y + s2 * d2.y;
  i2.x = s2 * d1.x - s1 * d2.x;
  i2.y = s2 * d1.y - s1 * d2.y;
  i1 = cmuli(i1);
  i2 = cmuli(i2);
  a[0] = y0;
  a[1] = cadd(r1, i1);
  a[4] = csub(r1, i1);
  a[2] = cadd(r2, i2);
  a[3] = csub(r2, i2);
}

template <typename T2>
__device__ __forceinline__ void dft8(T2* a) {
  using R = decltype(a[0].x);
  const R h = (R)0.70710678118654752440084436210485;
  T2 e[4] = {a[0], a[2], a[4], a[6]};
  T2 o[4] = {a[1], a[3], a[5], a[7]};
  dft4(e);
  dft4(o);
  // o_k *= w8^k, w8 = exp(2 pi i / 8)
  T2 o1, o2, o3;
  o1.x = h * (o[1].x - o[1].y);
  o1.y = h * (o[1].x + o[1].y);
  o2 = cmuli(o[2]);
  o3.x = -h * (o[3].x + o[3].y);
  o3.y = h * (o[3].x - o[3].y);
  a[0] = cadd(e[0], o[0]);
  a[4] = csub(e[0], o[0]);
  a[1] = cadd(e[1], o1);
  a[5] = csub(e[1], o1);
  a[2] = cadd(e[2], o2);
  a[6] = csub(e[2], o2);
  a[3] = cadd(e[3], o3);
  a[7] = csub(e[3], o3);
}

// 16 = 4 x 4: DFT4 over n1 of x[4 n1 + n2] for each n2, twiddles
// exp(+2 pi i n2 k1 / 16), then DFT4 over n2; output k1 + 4 k2.
template <typename T2>
__device__ __forceinline__ void dft16(T2* a) {
  using R = decltype(a[0].x);
  const R c1 = (R)0.92387953251128675612818318939679;  // cos(pi / 8)
  const R s1 = (R)0.38268343236508977172845998403040;  // sin(pi / 8)
  const R h = (R)0.70710678118654752440084436210485;
  T2 y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    T2 t[4] = {a[n2], a[n2 + 4], a[n2 + 8], a[n2 + 12]};
    dft4(t);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
  }
  // exp(+2 pi i j / 16) for j = n2 k1 in {1, 2, 3, 4, 6, 9}
  auto rot = [&](T2 v, R c, R s) {
    T2 r;
    r.x = v.x * c - v.y * s;
    r.y = v.x * s + v.y * c;
    return r;
  };
  auto rot45 = [&](T2 v) {  // j = 2
    T2 r;
    r.x = h * (v.x - v.y);
    r.y = h * (v.x + v.y);
    return r;
  };
  auto rot135 = [&](T2 v) {  // j = 6
    T2 r;
    r.x = -h * (v.x + v.y);
    r.y = h * (v.x - v.y);
    return r;
  };
  y[1][1] = rot(y[1][1], c1, s1);
  y[1][2] = rot45(y[1][2]);
  y[1][3] = rot(y[1][3], s1, c1);
  y[2][1] = rot45(y[2][1]);
  y[2][2] = cmuli(y[2][2]);
  y[2][3] = rot135(y[2][3]);
  y[3][1] = rot(y[3][1], s1, c1);
  y[3][2] = rot135(y[3][2]);
  y[3][3] = rot(y[3][3], -c1, -s1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    T2 t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    dft4(t);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[k2];
  }
}

template <int R, typename T2>
__device__ __forceinline__ void dft(T2* a) {
  if constexpr (R == 2) dft2(a);
  else if constexpr (R == 3) dft3(a);
  else if constexpr (R == 4) dft4(a);
  else if constexpr (R == 5) dft5(a);
  else if constexpr (R == 8) dft8(a);
  else if constexpr (R == 16) dft16(a);
}

// Quotient floor(j / d) for 0 <= j < 2048, 1 <= d <= 1024, given
// r = fdiv_recip(d): a float product and a truncation (exact over that range
// even with the reciprocal 2 ulp off; checked exhaustively on the host).
__device__ __forceinline__ float fdiv_recip(int d) {
  return __builtin_amdgcn_rcpf((float)d) * 1.000244140625f;
}
__device__ __forceinline__ int fdiv_small(int j, float r) { return (int)((float)j * r); }

// exp(2 pi i x / L) from the pass's LDS table: the full table, or (TW2) the
// two-level one, lo[x mod kTwLo] * hi[x / kTwLo] with hi after the kTwLo lo.
template <bool TW2, typename T2>
__device__ __forceinline__ T2 tw_at(const T2* tw, int x) {
  static_assert(kTwLo == 64, "two-level split by 6 bits");
  if constexpr (TW2) return cmul(tw[kTwLo + (x >> 6)], tw[x & (kTwLo - 1)]);
  else return tw[x];
}

// Per-thread walk over the butterflies (or elements) idx = tid + b*NT of a
// set of ncol columns, idx = j*ncol + col: the first (j, col) takes one
// division, each later one a few adds (NT = qn*ncol + rn with rn < ncol).
struct ColWalk {
  int j, col, qn, rn, ncol;
  __device__ __forceinline__ ColWalk(int tid, int nt, int nc) : ncol(nc) {
    j = tid / nc;
    col = tid - j * nc;
    qn = nt / nc;
    rn = nt - qn * nc;
  }
  __device__ __forceinline__ void next() {
    col += rn;
    j += qn;
    if (col >= ncol) {
      col -= ncol;
      ++j;
    }
  }
};

// One Stockham stage of radix R over `ncol` columns of length L held in LDS;
// element l of column c sits at buf[c + l*ls] (ls >= ncol).  Ns = product of
// the radices of the earlier stages.  twL[x] = exp(2 pi i x / L).  A thread
// takes butterflies j of column col as given by the walk (consecutive threads:
// consecutive columns of one butterfly, so the R reads and writes of a wave
// are runs of ncol contiguous elements).  All index arithmetic is 32-bit with
// 24-bit products: L <= 1024 and ls * L fits easily.
template <int R, int MAXB, int NT, bool TW2, typename T2>
__device__ __forceinline__ void stockham_stage(T2* buf, int L, int ls, int Ns, const T2* twL,
                                               ColWalk w) {
  const int nb = L / R;
  const int twstride = L / (Ns * R);
  const float rNs = fdiv_recip(Ns);
  const int rstep = nb * ls;       // between the R inputs of a butterfly
  const int wstep = Ns * ls;       // between its R outputs
  T2 v[MAXB][R];
  int wofs[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    wofs[b] = -1;
    if (w.j < nb) {
      const int jq = fdiv_small(w.j, rNs);
      const int k = w.j - __mul24(jq, Ns);
      const int rofs = w.col + __mul24(w.j, ls);
#pragma unroll
      for (int q = 0; q < R; ++q) v[b][q] = buf[rofs + q * rstep];
      if (Ns > 1) {
        const int kt = __mul24(k, twstride);
#pragma unroll
        for (int q = 1; q < R; ++q) v[b][q] = cmul(v[b][q], tw_at<TW2>(twL, q * kt));
      }
      dft<R>(v[b]);
      wofs[b] = w.col + __mul24(__mul24(jq, Ns * R) + k, ls);
    }
    w.next();
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    if (wofs[b] >= 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) buf[wofs[b] + q * wstep] = v[b][q];
    }
  }
  __syncthreads();
}

// Full transform of the ncol columns: runs the stages of the radix plan.
// EMAX bounds L * ncol (it sizes the per-thread register arrays); TW2 selects
// the two-level twiddle table.
template <int EMAX, int NT, bool TW2 = false, typename T2>
__device__ __forceinline__ void lds_fft(T2* buf, int L, int ncol, int ls, const int* rad, int nrad,
                        const T2* twL) {
  const ColWalk w(threadIdx.x, NT, ncol);
  int Ns = 1;
  for (int s = 0; s < nrad; ++s) {
    int r = rad[s];
    switch (r) {
      case 2:
        stockham_stage<2, (EMAX / 2 + NT - 1) / NT, NT, TW2>(buf, L, ls, Ns, twL, w);
        break;
      case 3:
        stockham_stage<3, (EMAX / 3 + NT - 1) / NT, NT, TW2>(buf, L, ls, Ns, twL, w);
        break;
      case 4:
        stockham_stage<4, (EMAX / 4 + NT - 1) / NT, NT, TW2>(buf, L, ls, Ns, twL, w);
        break;
      case 5:
        stockham_stage<5, (EMAX / 5 + NT - 1) / NT, NT, TW2>(buf, L, ls, Ns, twL, w);
        break;
      case 8:
        stockham_stage<8, (EMAX / 8 + NT - 1) / NT, NT, TW2>(buf, L, ls, Ns, twL, w);
        break;
      default:
        stockham_stage<16, (EMAX / 16 + NT - 1) / NT, NT, TW2>(buf, L, ls, Ns, twL, w);
        break;
    }
    Ns *= r;
  }
}

}  // namespace mils
