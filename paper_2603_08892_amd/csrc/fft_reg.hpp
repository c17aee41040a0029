// fft_reg.hpp -- compile-time register FFTs for the specialised passes (gfx950).
//
// A line of N points is shared by TPL threads, EPT = N / TPL points each.  The
// transform is a self-sorting Stockham FFT with a compile-time radix list: in a
// stage of radix R after Ns points have been combined, thread t computes the
// butterflies j = t + TPL b (b < EPT/R): points j + m N/R, twiddles W_N^{(j mod Ns) m},
// an R-point DFT, outputs to (j div Ns) Ns R + (j mod Ns) + m Ns.  Stages
// exchange points through LDS; the R-point DFTs run on registers.  After the
// last stage thread t holds the outputs t + TPL b + m N/R_last, which are the
// inputs of its first stage of a transform whose radix list starts with
// R_last, so an inverse transform can feed a forward one without an exchange.
//
// A stage of radix R has N/R butterflies; thread t takes butterflies
// t + TPL b, b < ceil(N / (R TPL)), and where TPL does not divide N/R the last ones
// are predicated off (a plan whose radices do not all divide one points-per-thread
// count, e.g. 240 = 10 4 6 over 24 threads).  EPT is then the most points a thread
// holds in any stage, and the first and last stages say which of its registers hold
// points (in_ok, out_ok).
//
// Composite DFTs (6, 9, 10, 12, 16, 24, 32) use the Cooley-Tukey split with
// compile-time twiddles; their cos/sin are evaluated at compile time from the
// Taylor series of the reduced angle.
#pragma once

#include "fft_core.hpp"

namespace ns {

// ---------------------------------------------------------------- compile-time cos/sin
constexpr long double ct_pi = 3.141592653589793238462643383279502884L;

constexpr long double ct_sin_series(long double x) {  // |x| <= pi/4
  long double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr long double ct_cos_series(long double x) {
  long double term = 1, sum = 1;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi num / den, exact octant reduction on the integer ratio
constexpr long double ct_cos2pi(long long num, long long den) {
  num %= den;
  if (num < 0) num += den;
  // angle = 2 pi num/den in [0, 2pi); reduce with 8*num vs den
  const long long e = 8 * num;  // octant index = floor(e / den)
  const int oct = (int)(e / den);
  const long double r = (long double)(e - (long long)oct * den) / (long double)den;  // in [0,1)
  const long double a = r * ct_pi / 4;  // residual angle in [0, pi/4)
  const long double c = ct_cos_series(a), s = ct_sin_series(a);
  const long double h = 0.70710678118654752440084436210484903928L;
  switch (oct) {  // cos(oct*pi/4 + a)
    case 0: return c;
    case 1: return h * (c - s);
    case 2: return -s;
    case 3: return -h * (c + s);
    case 4: return -c;
    case 5: return -h * (c - s);
    case 6: return s;
    default: return h * (c + s);
  }
}
constexpr long double ct_sin2pi(long long num, long long den) {
  return ct_cos2pi(4 * num - den, 4 * den);  // sin x = cos(x - pi/2)
}

// cos and sin of 2 pi t / R for t < R, tabulated at compile time (a constexpr
// variable is evaluated by the compiler; indexed with unrolled loop counters the
// entries fold into immediates)
template <int R>
struct CtTable {
  double c[R], s[R];
};
template <int R>
constexpr CtTable<R> make_ct_table() {
  CtTable<R> tab{};
  for (int t = 0; t < R; ++t) {
    tab.c[t] = (double)ct_cos2pi(t, R);
    tab.s[t] = (double)ct_sin2pi(t, R);
  }
  return tab;
}

// ---------------------------------------------------------------- register DFTs
template <int R, int S, typename T>
__device__ __forceinline__ void rdft(Cx<T>* a);

// Cooley-Tukey split R = A * B on registers: n = B n1 + n2, k = k1 + A k2.
template <int A, int B, int S, typename T>
__device__ __forceinline__ void rdft_split(Cx<T>* a) {
  constexpr int R = A * B;
  constexpr CtTable<R> tab = make_ct_table<R>();
  Cx<T> y[A][B];
#pragma unroll
  for (int n2 = 0; n2 < B; ++n2) {
    Cx<T> col[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) col[n1] = a[B * n1 + n2];
    rdft<A, S>(col);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      if (n2 * k1 == 0) {
        y[k1][n2] = col[k1];
      } else {
        const T c = T(tab.c[(n2 * k1) % R]);
        const T s = T(S * tab.s[(n2 * k1) % R]);
        y[k1][n2] = cx(col[k1].re * c - col[k1].im * s, col[k1].re * s + col[k1].im * c);
      }
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    rdft<B, S>(y[k1]);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) a[k1 + A * k2] = y[k1][k2];
  }
}

template <int R, int S, typename T>
__device__ __forceinline__ void rdft(Cx<T>* a) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) dft2<S>(a);
  else if constexpr (R == 3) dft3<S>(a);
  else if constexpr (R == 4) dft4<S>(a);
  else if constexpr (R == 5) dft5<S>(a);
  else if constexpr (R == 8) dft8<S>(a);
  else if constexpr (R == 6) rdft_split<2, 3, S>(a);
  else if constexpr (R == 9) rdft_split<3, 3, S>(a);
  else if constexpr (R == 10) rdft_split<2, 5, S>(a);
  else if constexpr (R == 12) rdft_split<4, 3, S>(a);
  else if constexpr (R == 16) rdft_split<4, 4, S>(a);
  else if constexpr (R == 24) rdft_split<8, 3, S>(a);
  else if constexpr (R == 32) rdft_split<4, 8, S>(a);
  else static_assert(R == 2, "unsupported register DFT size");
}

// ---------------------------------------------------------------- LDS views of a line
// Point `pos` of the line at base[pos * ES] (ES > 1: lines interleaved with pitch
// ES), or, for ES == 1 (contiguous lines), at base[pos + pos / 16]: one padding
// element every 16 points so that the stride-R writes of the early stages spread
// over the LDS banks.
template <typename T, int ES>
struct LineView {
  Cx<T>* base;
  __device__ __forceinline__ Cx<T>& at(int pos) const {
    if constexpr (ES == 1) return base[pos + (pos >> 4)];
    else return base[pos * ES];
  }
};
// LDS elements of one contiguous line of n points in the ES == 1 layout
__host__ __device__ constexpr int line_pitch(int n) { return n + n / 16 + 1; }

// Stages of one transform on the registers v[b * R + m] (b < EPT/R) of thread t.
// NS = points already combined.  Twiddles from the table tw[] (W_N^t, t < N).
// Each exchange: barrier, write, barrier, read (the buffer may still be read by
// the previous use, so the first barrier is kept).  WAVE: all TPL threads of a
// line are in one wavefront, whose LDS operations complete in program order, so
// the barriers only have to order the LDS accesses at wavefront scope (fences
// around a wavefront barrier) instead of synchronising the whole block.
template <bool WAVE>
__device__ __forceinline__ void exchange_barrier() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Butterflies per thread of a stage of radix R, and whether all of them are real.
template <int N, int TPL, int R>
struct StageMap {
  static constexpr int NB = (N / R + TPL - 1) / TPL;
  static constexpr bool FULL = (N / R) % TPL == 0;
  __device__ __forceinline__ static bool ok(int t, int b) { return FULL || t + TPL * b < N / R; }
};

template <int N, int TPL, int S, int NS, int R, int... Rest>
struct RegStages {
  template <bool WAVE, typename T, int ES>
  __device__ __forceinline__ static void run(Cx<T>* v, int t, const LineView<T, ES>& lv, const Cx<T>* tw) {
    using M = StageMap<N, TPL, R>;
    constexpr int NB = M::NB;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (!M::ok(t, b)) continue;
      const int j = t + TPL * b;
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int m = 1; m < R; ++m) {
          const Cx<T> w = tw[k * m * (N / (NS * R))];
          v[b * R + m] = (S < 0) ? cmul(v[b * R + m], w) : cmulc(v[b * R + m], w);
        }
      }
      rdft<R, S>(v + b * R);
    }
    if constexpr (sizeof...(Rest) > 0) {
      constexpr int R2 = first_of<Rest...>();
      using M2 = StageMap<N, TPL, R2>;
      constexpr int NB2 = M2::NB;
      exchange_barrier<WAVE>();
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (!M::ok(t, b)) continue;
        const int j = t + TPL * b;
        const int k = j % NS, q = j / NS;
#pragma unroll
        for (int m = 0; m < R; ++m) lv.at(q * NS * R + k + m * NS) = v[b * R + m];
      }
      exchange_barrier<WAVE>();
#pragma unroll
      for (int b = 0; b < NB2; ++b) {
        if (!M2::ok(t, b)) continue;
        const int j = t + TPL * b;
#pragma unroll
        for (int m = 0; m < R2; ++m) v[b * R2 + m] = lv.at(j + m * (N / R2));
      }
      RegStages<N, TPL, S, NS * R, Rest...>::template run<WAVE>(v, t, lv, tw);
    }
  }
  template <int F, int... X>
  static constexpr int first_of() { return F; }
};

template <int... Rs>
struct Radices {
  static constexpr int count = sizeof...(Rs);
  // most points a thread holds in any stage of an N-point transform over TPL threads
  template <int N, int TPL>
  static constexpr int ept() {
    int e = 0;
    for (int r : {Rs...}) {
      const int v = (N / r + TPL - 1) / TPL * r;
      e = v > e ? v : e;
    }
    return e;
  }
  // every stage gives every thread the same number of whole butterflies
  template <int N, int TPL>
  static constexpr bool uniform() {
    bool u = true;
    for (int r : {Rs...}) u = u && (N / r) % TPL == 0 && (N / r) / TPL * r == N / TPL;
    return u;
  }
  static constexpr int first() { return first_impl<Rs...>(); }
  static constexpr int last() { return last_impl<Rs...>(); }
  static constexpr int product() { return (Rs * ...); }
  template <int F, int... X>
  static constexpr int first_impl() { return F; }
  template <int F, int... X>
  static constexpr int last_impl() {
    if constexpr (sizeof...(X) == 0) return F;
    else return last_impl<X...>();
  }
};

template <int N, int TPL, int S, typename Rad>
struct RegFft;
template <int N, int TPL, int S, int... Rs>
struct RegFft<N, TPL, S, Radices<Rs...>> {
  using Rad = Radices<Rs...>;
  static constexpr int EPT = Rad::template ept<N, TPL>();
  static constexpr bool UNIFORM = Rad::template uniform<N, TPL>();
  static constexpr int R0 = Rad::first();
  static constexpr int RL = Rad::last();
  static_assert(Rad::product() == N, "radices must multiply to N");
  // input position of register i (i = b * R0 + m) of thread t before the first stage
  __device__ __forceinline__ static int in_pos(int t, int i) { return t + TPL * (i / R0) + (i % R0) * (N / R0); }
  // output position of register i (i = b * RL + m) of thread t after the last stage
  __device__ __forceinline__ static int out_pos(int t, int i) { return t + TPL * (i / RL) + (i % RL) * (N / RL); }
  // whether register i of thread t holds a point before the first / after the last
  // stage (always, for a uniform plan); the positions of other registers are not
  // points of the line and must not address memory
  __device__ __forceinline__ static bool in_ok(int t, int i) {
    if constexpr (UNIFORM) return true;
    else return i / R0 < StageMap<N, TPL, R0>::NB && StageMap<N, TPL, R0>::ok(t, i / R0);
  }
  __device__ __forceinline__ static bool out_ok(int t, int i) {
    if constexpr (UNIFORM) return true;
    else return i / RL < StageMap<N, TPL, RL>::NB && StageMap<N, TPL, RL>::ok(t, i / RL);
  }
  // the positions with a stand-in 0 for registers that hold no point, for indexing
  // tables of the line (the value of such a register is never used)
  __device__ __forceinline__ static int in_at(int t, int i) { return in_ok(t, i) ? in_pos(t, i) : 0; }
  __device__ __forceinline__ static int out_at(int t, int i) { return out_ok(t, i) ? out_pos(t, i) : 0; }
  template <bool WAVE = false, typename T, int ES>
  __device__ __forceinline__ static void run(Cx<T>* v, int t, const LineView<T, ES>& lv, const Cx<T>* tw) {
    static_assert(!WAVE || TPL <= 64, "a wavefront-local line fits in one wavefront");
    RegStages<N, TPL, S, 1, Rs...>::template run<WAVE>(v, t, lv, tw);
  }
};

}  // namespace ns
