// fft_core.hpp -- device building blocks of the pencil FFT passes (gfx950).
//
// A pass transforms many lines of length N that sit in LDS.  Each stage of a
// mixed-radix Stockham (self-sorting) FFT reads R points x[j + m N/R] of every
// butterfly j, multiplies point m by W^(k m), k = j mod Ns (Ns = product of the
// radices already applied), runs an R-point DFT and writes point m to
// (j div Ns) Ns R + k + m Ns.  All threads read their butterflies into registers,
// the block synchronises, then all threads write: one LDS buffer per line set.
//
// Twiddles come from a table W_N^t = exp(-2 pi i t / N), t < N, generated in
// long double on the host and rounded once to the field type; the inverse
// direction uses the conjugates.  Butterfly constants are exact decimal
// expansions of cos/sin of multiples of 2 pi/3, 2 pi/5, 2 pi/8.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ns {

template <typename R>
struct __attribute__((aligned(2 * sizeof(R)))) Cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ Cx<R> cx(R a, R b) { Cx<R> z; z.re = a; z.im = b; return z; }
template <typename R>
__device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return cx(a.re + b.re, a.im + b.im); }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return cx(a.re - b.re, a.im - b.im); }
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return cx(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {  // a * conj(b)
  return cx(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
template <typename R>
__device__ __forceinline__ Cx<R> conj(Cx<R> a) { return cx(a.re, -a.im); }
template <typename R>
__device__ __forceinline__ Cx<R> scale(Cx<R> a, R s) { return cx(a.re * s, a.im * s); }
// multiply by s*i, s = +1 or -1
template <int S, typename R>
__device__ __forceinline__ Cx<R> mul_si(Cx<R> a) {
  return S > 0 ? cx(-a.im, a.re) : cx(a.im, -a.re);
}

constexpr double kSqrt3_2 = 0.86602540378443864676372317075294;   // sin(2 pi/3)
constexpr double kRsqrt2 = 0.70710678118654752440084436210485;    // cos(pi/4)
constexpr double kC5_1 = 0.30901699437494742410229341718282;      // cos(2 pi/5)
constexpr double kC5_2 = -0.80901699437494742410229341718282;     // cos(4 pi/5)
constexpr double kS5_1 = 0.95105651629515357211643933337938;      // sin(2 pi/5)
constexpr double kS5_2 = 0.58778525229247312916870595463907;      // sin(4 pi/5)

// R-point DFTs y_k = sum_m a_m exp(S 2 pi i k m / R), S = -1 forward, +1 inverse.
template <int S, typename R>
__device__ __forceinline__ void dft2(Cx<R>* a) {
  Cx<R> t = a[0];
  a[0] = t + a[1];
  a[1] = t - a[1];
}

template <int S, typename R>
__device__ __forceinline__ void dft3(Cx<R>* a) {
  Cx<R> t1 = a[1] + a[2];
  Cx<R> t2 = a[0] - scale(t1, R(0.5));
  Cx<R> t3 = mul_si<S>(scale(a[1] - a[2], R(kSqrt3_2)));
  a[0] = a[0] + t1;
  a[1] = t2 + t3;
  a[2] = t2 - t3;
}

template <int S, typename R>
__device__ __forceinline__ void dft4(Cx<R>* a) {
  Cx<R> s02 = a[0] + a[2], d02 = a[0] - a[2];
  Cx<R> s13 = a[1] + a[3], d13 = mul_si<S>(a[1] - a[3]);
  a[0] = s02 + s13;
  a[2] = s02 - s13;
  a[1] = d02 + d13;
  a[3] = d02 - d13;
}

template <int S, typename R>
__device__ __forceinline__ void dft5(Cx<R>* a) {
  Cx<R> t1 = a[1] + a[4], t2 = a[2] + a[3];
  Cx<R> t3 = a[1] - a[4], t4 = a[2] - a[3];
  Cx<R> b1 = a[0] + scale(t1, R(kC5_1)) + scale(t2, R(kC5_2));
  Cx<R> b2 = a[0] + scale(t1, R(kC5_2)) + scale(t2, R(kC5_1));
  Cx<R> d1 = mul_si<S>(scale(t3, R(kS5_1)) + scale(t4, R(kS5_2)));
  Cx<R> d2 = mul_si<S>(scale(t3, R(kS5_2)) - scale(t4, R(kS5_1)));
  a[0] = a[0] + t1 + t2;
  a[1] = b1 + d1;
  a[4] = b1 - d1;
  a[2] = b2 + d2;
  a[3] = b2 - d2;
}

template <int S, typename R>
__device__ __forceinline__ void dft8(Cx<R>* a) {
  Cx<R> e[4] = {a[0], a[2], a[4], a[6]};
  Cx<R> o[4] = {a[1], a[3], a[5], a[7]};
  dft4<S>(e);
  dft4<S>(o);
  const R r = R(kRsqrt2);
  // w^k = exp(S 2 pi i k / 8)
  Cx<R> o1 = scale(o[1] + mul_si<S>(o[1]), r);        // (1 + S i)/sqrt2
  Cx<R> o2 = mul_si<S>(o[2]);                          // S i
  Cx<R> o3 = scale(mul_si<S>(o[3]) - o[3], r);        // (-1 + S i)/sqrt2
  a[0] = e[0] + o[0];
  a[4] = e[0] - o[0];
  a[1] = e[1] + o1;
  a[5] = e[1] - o1;
  a[2] = e[2] + o2;
  a[6] = e[2] - o2;
  a[3] = e[3] + o3;
  a[7] = e[3] - o3;
}

template <int RAD, int S, typename R>
__device__ __forceinline__ void dft(Cx<R>* a) {
  if constexpr (RAD == 2) dft2<S>(a);
  else if constexpr (RAD == 3) dft3<S>(a);
  else if constexpr (RAD == 4) dft4<S>(a);
  else if constexpr (RAD == 5) dft5<S>(a);
  else dft8<S>(a);
}

// FFT plan of one length: the radix sequence and, per stage, Ns and N/(Ns R).
constexpr int kMaxStages = 12;
struct FftPlan {
  int n;
  int nstages;
  int radix[kMaxStages];
  int ns[kMaxStages];
  int tstride[kMaxStages];
};

// Lines in LDS: point p of line l at buf[p * pstride + l * lstride].
// LINE_FAST = true: consecutive threads take consecutive lines of the same
// butterfly index (the [p][l] layout of the strided passes); false: consecutive
// butterfly indices of one line (the [l][p] layout of the contiguous pass).
template <int RAD, int S, int NB, bool LINE_FAST, typename R>
__device__ __forceinline__ void fft_stage(Cx<R>* buf, const Cx<R>* tw, int n, int ns, int tstride,
                                          int nlines, int pstride, int lstride, int tid,
                                          int nthreads) {
  const int nbl = n / RAD;  // butterflies per line
  const int total = nbl * nlines;
  const int quarter = n / RAD;
  Cx<R> v[NB][RAD];
  int obase[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int bi = tid + b * nthreads;
    obase[b] = -1;
    if (bi < total) {
      int l, j;
      if (LINE_FAST) { l = bi % nlines; j = bi / nlines; }
      else { j = bi % nbl; l = bi / nbl; }
      const int k = j % ns;
      const int q = j / ns;
      const Cx<R>* src = buf + l * lstride;
#pragma unroll
      for (int m = 0; m < RAD; ++m) v[b][m] = src[(j + m * quarter) * pstride];
      if (ns > 1) {
#pragma unroll
        for (int m = 1; m < RAD; ++m) {
          Cx<R> w = tw[k * m * tstride];
          v[b][m] = (S < 0) ? cmul(v[b][m], w) : cmulc(v[b][m], w);
        }
      }
      dft<RAD, S>(v[b]);
      obase[b] = (q * ns * RAD + k) * pstride + l * lstride;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (obase[b] >= 0) {
#pragma unroll
      for (int m = 0; m < RAD; ++m) buf[obase[b] + m * ns * pstride] = v[b][m];
    }
  }
  __syncthreads();
}

// Whole FFT of `nlines` lines in LDS.  EPT bounds the points per thread:
// n * nlines <= EPT * nthreads.  Ends synchronised.
template <int S, int EPT, bool LINE_FAST, typename R>
__device__ void fft_lines(Cx<R>* buf, const Cx<R>* tw, const FftPlan& plan, int nlines,
                          int pstride, int lstride, int tid, int nthreads) {
  for (int s = 0; s < plan.nstages; ++s) {
    const int rad = plan.radix[s], ns = plan.ns[s], ts = plan.tstride[s];
    switch (rad) {
      case 8: fft_stage<8, S, (EPT + 7) / 8, LINE_FAST>(buf, tw, plan.n, ns, ts, nlines, pstride, lstride, tid, nthreads); break;
      case 4: fft_stage<4, S, (EPT + 3) / 4, LINE_FAST>(buf, tw, plan.n, ns, ts, nlines, pstride, lstride, tid, nthreads); break;
      case 2: fft_stage<2, S, (EPT + 1) / 2, LINE_FAST>(buf, tw, plan.n, ns, ts, nlines, pstride, lstride, tid, nthreads); break;
      case 3: fft_stage<3, S, (EPT + 2) / 3, LINE_FAST>(buf, tw, plan.n, ns, ts, nlines, pstride, lstride, tid, nthreads); break;
      default: fft_stage<5, S, (EPT + 4) / 5, LINE_FAST>(buf, tw, plan.n, ns, ts, nlines, pstride, lstride, tid, nthreads); break;
    }
  }
}

}  // namespace ns
