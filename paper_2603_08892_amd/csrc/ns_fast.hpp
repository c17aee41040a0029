// ns_fast.hpp -- compile-time specialised passes for the common grid sizes (FP32, gfx950).
//
// Same scratch layout, tile list and pass semantics as the generic kernels of
// ns_kernels.hpp, except that in the step sequences the x-inverse passes store
// the five transforms they compute and the y-inverse pass (f_ycurl) forms the
// vorticity from them; the transforms run on registers (fft_reg.hpp) with one LDS
// exchange per radix boundary instead of one LDS round trip per stage, and all
// indices are compile-time except the thread and block coordinates.
//
// Strided passes (x, y): a block is one tile of L = 16 contiguous k_z columns;
// thread (l, t) = (tid mod L, tid div L) handles column l, points of the line
// owned by t.  LDS: the exchange buffer [position][column] (row pitch L + 1 to
// spread banks) and the twiddle table.
// Contiguous pass (z): a block holds P lines, thread (p, t) = (tid div TPL, tid mod TPL);
// a line's threads synchronise at wavefront scope when TPL divides 64 (every z plan
// below) and with block barriers otherwise.
// In the step sequences the x-forward kernel can also run the next evaluation's
// x-inverse pass on its tile (template argument FEED), so a chained evaluation is
// four launches: y-inverse, z, y-forward, x-forward (+ next x-inverse).
#pragma once

#include "fft_reg.hpp"
#include "ns_kernels.hpp"

namespace ns {

constexpr int kFastL = 16;
constexpr int kFastLp = kFastL + 1;

// Addressing: a block-uniform base pointer (a state component or scratch field)
// plus a per-lane 32-bit element offset.  Every offset stays inside one component
// of at most N^2 (N/2 + 1) elements, and the specialised sizes keep 8 bytes times
// that below 2^32 (FastCfg checks it), so the byte offset fits 32 bits, the base
// stays in scalar registers and the index arithmetic is 32-bit.
__device__ __forceinline__ Cx<float> ld_off(const Cx<float>* __restrict__ base, uint32_t off) {
  return *reinterpret_cast<const Cx<float>*>(reinterpret_cast<const char*>(base) + off * 8u);
}
// STREAM: a non-temporal store, for the scratch fields and the compact stage
// buffers of the grids whose step works on far more than the 256 MB last-level
// cache (stream_stores): each pass's output is read back only by the next pass,
// mostly on other XCDs, so keeping it in cache buys nothing.  Measured per step
// (PS-RK2 random, RK4 at 512): 3-11% faster at N = 240...512, 256 gaining least;
// at N <= 216 much of a step's data is still found in that cache and the step
// was 5-17% slower.  Outputs in the
// caller's layout (rows of N/2 + 1 elements, not whole 128-byte lines) take
// plain stores: streamed partial lines made those passes 1.5 times slower.
constexpr bool stream_stores(int n) { return n >= 240; }
template <bool STREAM = false>
__device__ __forceinline__ void st_off(Cx<float>* __restrict__ base, uint32_t off, Cx<float> v) {
  if constexpr (STREAM) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 w = {v.re, v.im};
    __builtin_nontemporal_store(w, reinterpret_cast<f2*>(reinterpret_cast<char*>(base) + off * 8u));
  } else {
    *reinterpret_cast<Cx<float>*>(reinterpret_cast<char*>(base) + off * 8u) = v;
  }
}

// Branch-free masked load: the offset is clamped to element 0 of the (valid)
// base when `ok` is false and the value multiplied by 0 (the arrays hold finite
// values), so the load is unconditional and a thread issues all of its loads back
// to back before the first use (a select would let the compiler turn the load
// back into a branch with a wait right behind it).
__device__ __forceinline__ Cx<float> ld_masked(const Cx<float>* __restrict__ base, uint32_t off, bool ok) {
  const Cx<float> v = ld_off(base, ok ? off : 0u);
  const float m = ok ? 1.f : 0.f;
  return cx(v.re * m, v.im * m);
}

// Truncation test along one k_x line (fixed k_y, k_z) in 32-bit arithmetic
// (|k_i| <= N/2 <= 256 here, so |k|^2 < 2^18): every mask is k_x^2 <= hi2 and
// |k_x| <= xmax with per-line thresholds (xmax from the pair conditions of
// double_alias_free).
struct LineTest {
  int hi2, xmax;
  __device__ __forceinline__ bool operator()(int kx) const {
    // evaluated without short-circuit branches, so masked loads stay unconditional
    return (kx * kx <= hi2) & (abs(kx) <= xmax);
  }
};
__device__ __forceinline__ LineTest line_test(const Geom& g, int ky, int kz) {
  LineTest L{0, g.n};
  if (cube_family(g)) L.hi2 = (abs(ky) <= g.kmax && kz <= g.kmax) ? g.kmax * g.kmax : -1;
  else L.hi2 = (int)g.k2max - ky * ky - kz * kz;
  if (g.mask >= 2) {
    // 3 (|k_x| + |k_y|) < 2N, 3 (|k_x| + |k_z|) < 2N and 3 (|k_y| + |k_z|) < 2N
    const int b = abs(ky), c = abs(kz), n2 = 2 * g.n;
    L.xmax = (3 * (b + c) < n2) ? (n2 - 1) / 3 - max(b, c) : -1;
  }
  return L;
}

// Shift factors of the block's 16 k_z columns on row k_y (FP64, rounded once per
// axis like phase1), computed by 16 threads into LDS.
__device__ __forceinline__ void phase_cols(Cx<float>* phc, int ky, int kz0, const Shift& sh, int n, int tid) {
  if (tid < kFastL) phc[tid] = cmul(phase1<float>(ky, sh.s[1], n), phase1<float>(kz0 + tid, sh.s[2], n));
}

// One line plan: N points over TPL threads, inverse and forward radix lists.
template <int N_, int TPL_, typename Inv_, typename Fwd_>
struct LinePlan {
  static constexpr int N = N_;
  static constexpr int TPL = TPL_;
  static constexpr int EPT = Inv_::template ept<N_, TPL_>();
  static_assert(EPT == Fwd_::template ept<N_, TPL_>(), "both directions hold the same registers");
  using Inv = Inv_;   // radices of the inverse transforms
  using Fwd = Fwd_;   // radices of the forward transforms (reverse order of Inv)
};

// Plans of the five passes of one size; PZ = lines per block of the z pass; the
// adjoint z pass (five inverse and three forward slices) may take its own plan ZA
// with PZA lines per block.  YC: the step sequences run f_xinv<XI, false> and
// f_ycurl (the vorticity formed in the y-inverse pass, five scratch fields written
// by the x-inverse passes) instead of f_xinv<XI, true> and f_ypass over six fields.
template <typename XI, typename YP, typename ZP, int PZ_, typename XF, typename ZA = ZP, int PZA_ = PZ_,
          bool YC_ = false>
struct FastCfg {
  static constexpr int N = XI::N;
  static constexpr bool YC = YC_;
  static_assert(8ull * N * N * (N / 2 + 1) < (1ull << 32), "32-bit byte offsets need 8 N^2 (N/2+1) < 2^32");
  static constexpr int PZ = PZ_;
  static constexpr int PZA = PZA_;
  static_assert(N * N % PZ_ == 0 && N * N % PZA_ == 0, "the z passes run N^2 / P blocks of P whole lines");
  using XInv = XI;
  using Y = YP;
  using Z = ZP;
  using ZAdj = ZA;
  using XFwd = XF;
};

// ------------------------------------------------------------------ x inverse
// One active tile per block, all six fields.  Along an x line k_y and k_z are
// fixed, so the x transform of omega_x = i (k_y u_z - k_z u_y) is
// i k_y X(u_z) - i k_z X(u_y), and omega_y = i k_z u_x - i k_x u_z,
// omega_z = i k_x u_y - i k_y u_x need only D_z = X(i k_x u_z) and D_y = X(i k_x u_y)
// beside the velocity transforms: five transforms for six fields, and each state
// component is read once per tile.
// CURL = true stores the vorticity itself (fields 0..5 = u_x, u_y, u_z, omega_x,
// omega_y, omega_z), as f_ypass reads it (the transposed evaluations and the sizes
// without FastCfg::YC).  CURL = false stores the five transforms as they are: u_x,
// u_y, u_z in fields 0, 1, 2, D_z in field 4 and D_y in field 5, and leaves field
// 3 alone; f_ycurl forms the vorticity from them as it loads them, so a tile
// writes five fields here and is read as five there instead of six.
template <typename C, bool CURL>
__global__ void __launch_bounds__(kFastL * C::TPL)
f_xinv(const Cx<float>* __restrict__ S, Lay ls, Cx<float>* __restrict__ W, const Cx<float>* __restrict__ twg,
        Shift sh, const int2* __restrict__ tiles, Geom g) {
  constexpr int N = C::N, TPL = C::TPL, EPT = C::EPT;
  using F = RegFft<N, TPL, +1, typename C::Inv>;
  __shared__ Cx<float> tw[N];
  __shared__ Cx<float> phx[N];
  __shared__ Cx<float> phc[kFastL];
  __shared__ Cx<float> xb[N * kFastLp];
  const int tid = threadIdx.x;
  const int l = tid % kFastL, t = tid / kFastL;
  const int2 tile = tiles[blockIdx.x];
  const int yi = tile.x, kz0 = tile.y, kz = kz0 + l;
  const int ky = kval(yi, N);
  for (int i = tid; i < N; i += kFastL * TPL) tw[i] = twg[i];
  const bool col = kz < g.kzn;
  Cx<float> phyz = cx(1.f, 0.f);
  if (sh.on) {
    phase_row(phx, N, sh.s[0], tid, kFastL * TPL);
    phase_cols(phc, ky, kz0, sh, N, tid);
    __syncthreads();
    phyz = phc[l];
  }
  const LineView<float, kFastLp> lv{xb + l};
  const uint32_t sbase = (uint32_t)(yi * ls.pitch + kz0) + l, sstep = (uint32_t)(N * ls.pitch);
  [[maybe_unused]] const float kyf = float(ky), kzf = float(kz);
  Cx<float> ux[EPT], uy[EPT], uz[EPT], dy[EPT], dz[EPT];
  {
    bool ok[EPT];
    uint32_t idx[EPT];
    const LineTest keep = line_test(g, ky, kz);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int p = F::in_at(t, i);
      ok[i] = col && F::in_ok(t, i) && keep(kval(p, N));
      idx[i] = (uint32_t)p * sstep + sbase;
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      ux[i] = ld_masked(S, idx[i], ok[i]);
      uy[i] = ld_masked(S + ls.cs, idx[i], ok[i]);
      uz[i] = ld_masked(S + 2 * ls.cs, idx[i], ok[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int p = F::in_at(t, i);
    if (sh.on) {
      const Cx<float> phi = cmul(phx[p], phyz);
      ux[i] = cmul(ux[i], phi);
      uy[i] = cmul(uy[i], phi);
      uz[i] = cmul(uz[i], phi);
    }
    const float kxf = float(kval(p, N));
    dy[i] = mul_i(scale(uy[i], kxf));
    dz[i] = mul_i(scale(uz[i], kxf));
  }
  const uint32_t obase = (uint32_t)(yi * g.kzp + kz0) + l, ostep = (uint32_t)(N * g.kzp);
  auto store = [&](int f, const Cx<float>* v) {
    if (col) {
#pragma unroll
      for (int i = 0; i < EPT; ++i)
        if (F::out_ok(t, i))
          st_off<stream_stores(N)>(W + f * g.wcomp, (uint32_t)F::out_pos(t, i) * ostep + obase, v[i]);
    }
  };
  F::run(uy, t, lv, tw);
  store(1, uy);
  F::run(uz, t, lv, tw);
  store(2, uz);
  if constexpr (CURL) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) uy[i] = mul_i(scale(uz[i], kyf) - scale(uy[i], kzf));  // omega_x
    store(3, uy);
  }
  F::run(ux, t, lv, tw);
  store(0, ux);
  F::run(dz, t, lv, tw);
  if constexpr (CURL) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) dz[i] = mul_i(scale(ux[i], kzf)) - dz[i];  // omega_y
  }
  store(4, dz);
  F::run(dy, t, lv, tw);
  if constexpr (CURL) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) dy[i] = dy[i] - mul_i(scale(ux[i], kyf));  // omega_z
  }
  store(5, dy);
}

// ------------------------------------------------------------------ y passes (in place)
template <typename C, int S>
__global__ void __launch_bounds__(kFastL * C::TPL)
f_ypass(Cx<float>* __restrict__ W, const Cx<float>* __restrict__ twg, int ntz, Geom g) {
  constexpr int N = C::N, TPL = C::TPL, EPT = C::EPT;
  using F = RegFft<N, TPL, S, std::conditional_t<(S > 0), typename C::Inv, typename C::Fwd>>;
  __shared__ Cx<float> tw[N];
  __shared__ Cx<float> xb[N * kFastLp];
  const int tid = threadIdx.x;
  const int l = tid % kFastL, t = tid / kFastL;
  const int b = blockIdx.x;
  const int kzt = b % ntz, rest = b / ntz;
  const int x = rest % N, f = rest / N;
  const int kz0 = kzt * kFastL, kz = kz0 + l;
  const int yb = ybound(g, kz0);
  for (int i = tid; i < N; i += kFastL * TPL) tw[i] = twg[i];
  const bool col = kz < g.kzn;
  Cx<float>* base = W + f * g.wcomp;
  const uint32_t rbase = (uint32_t)(x * N * g.kzp + kz0) + l;
  const LineView<float, kFastLp> lv{xb + l};
  Cx<float> v[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int p = F::in_at(t, i);
    v[i] = ld_masked(base, (uint32_t)(p * g.kzp) + rbase, col && F::in_ok(t, i) && (S < 0 || abs(kval(p, N)) <= yb));
  }
  F::run(v, t, lv, tw);
  if (col) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int p = F::out_pos(t, i);
      if (F::out_ok(t, i) && (S > 0 || abs(kval(p, N)) <= yb))
        st_off<stream_stores(N)>(base, (uint32_t)(p * g.kzp) + rbase, v[i]);
    }
  }
}

// ------------------------------------------------------------------ y inverse with the curl
// The y-inverse pass of the step sequences of the sizes with FastCfg::YC, after
// f_xinv<C, false> (or the fused x-forward pass), which stores u_x, u_y, u_z, D_z
// and D_y in scratch fields 0, 1, 2, 4, 5.  A point here has fixed k_y and k_z,
// so the vorticity is a pointwise combination of the stored transforms,
//   omega_x = i (k_y u_z - k_z u_y),  omega_y = i k_z u_x - D_z,  omega_z = D_y - i k_y u_x,
// formed in registers before the y transform.  Block group 0 reads u_y, u_z and
// writes u_y, u_z, omega_x (fields 1, 2, 3); group 1 reads u_x, D_z, D_y and writes
// u_x, omega_y, omega_z (fields 0, 4, 5).  Each field is read once; a block's
// loads all come before its stores and no other block touches its fields on its
// (x, k_z tile), so the pass runs in place.  Output as f_ypass<C, +1> over six
// fields.  Three line buffers a thread: at 12 points a thread or over more than
// 32 threads a line this allows one block per CU, where the six single-field
// blocks of f_ypass keep two or three resident and are faster.
template <typename C>
__global__ void __launch_bounds__(kFastL * C::TPL)
f_ycurl(Cx<float>* __restrict__ W, const Cx<float>* __restrict__ twg, int ntz, Geom g) {
  constexpr int N = C::N, TPL = C::TPL, EPT = C::EPT;
  using F = RegFft<N, TPL, +1, typename C::Inv>;
  __shared__ Cx<float> tw[N];
  __shared__ Cx<float> xb[N * kFastLp];
  const int tid = threadIdx.x;
  const int l = tid % kFastL, t = tid / kFastL;
  const int b = blockIdx.x;
  const int kzt = b % ntz, rest = b / ntz;
  const int x = rest % N, grp = rest / N;
  const int kz0 = kzt * kFastL, kz = kz0 + l;
  const int yb = ybound(g, kz0);
  for (int i = tid; i < N; i += kFastL * TPL) tw[i] = twg[i];
  const bool col = kz < g.kzn;
  Cx<float>* const Wa = W + (grp ? 0 : 1) * g.wcomp;
  Cx<float>* const Wb = W + (grp ? 4 : 2) * g.wcomp;
  Cx<float>* const Wc = W + (grp ? 5 : 3) * g.wcomp;
  const uint32_t rbase = (uint32_t)(x * N * g.kzp + kz0) + l;
  const LineView<float, kFastLp> lv{xb + l};
  Cx<float> va[EPT], vb[EPT], vc[EPT];
  {
    bool ok[EPT];
    uint32_t idx[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int p = F::in_at(t, i);
      ok[i] = col && F::in_ok(t, i) && abs(kval(p, N)) <= yb;
      idx[i] = (uint32_t)(p * g.kzp) + rbase;
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      va[i] = ld_masked(Wa, idx[i], ok[i]);
      vb[i] = ld_masked(Wb, idx[i], ok[i]);
    }
    if (grp) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) vc[i] = ld_masked(Wc, idx[i], ok[i]);
    }
  }
  const float kzf = float(kz);
  if (grp) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const float kyf = float(kval(F::in_at(t, i), N));
      vb[i] = mul_i(scale(va[i], kzf)) - vb[i];  // omega_y
      vc[i] = vc[i] - mul_i(scale(va[i], kyf));  // omega_z
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const float kyf = float(kval(F::in_at(t, i), N));
      vc[i] = mul_i(scale(vb[i], kyf) - scale(va[i], kzf));  // omega_x
    }
  }
  auto store = [&](Cx<float>* base, const Cx<float>* v) {
    if (col) {
#pragma unroll
      for (int i = 0; i < EPT; ++i)
        if (F::out_ok(t, i)) st_off<stream_stores(N)>(base, (uint32_t)(F::out_pos(t, i) * g.kzp) + rbase, v[i]);
    }
  };
  F::run(va, t, lv, tw);
  store(Wa, va);
  F::run(vb, t, lv, tw);
  store(Wb, vb);
  F::run(vc, t, lv, tw);
  store(Wc, vc);
}

// ------------------------------------------------------------------ z fused
// P lines per block.  Inverse slices (u_x + i u_y), (u_z + i w_x), (w_y + i w_z) built
// from the half spectra on the fly (Z(k) = a(k) + i b(k), Z(N-k) = conj a(k) + i conj b(k),
// imaginary parts of the k_z = 0 and N/2 coefficients dropped); the product
// f = u x omega stays in registers; forward slices (f_x + i f_y) and f_z; the
// spectra are split through LDS.  Output scratch fields 0, 1, 2 = f_x, f_y, f_z (unnormalised).
template <typename C, int P>
__global__ void __launch_bounds__(P * C::TPL)
f_zcross(Cx<float>* __restrict__ W, const Cx<float>* __restrict__ twg, Geom g) {
  constexpr int N = C::N, TPL = C::TPL, EPT = C::EPT, HN = N / 2, NT = P * TPL;
  using FI = RegFft<N, TPL, +1, typename C::Inv>;
  using FF = RegFft<N, TPL, -1, typename C::Fwd>;
  static_assert(FI::RL == FF::R0, "the forward transform must start with the last inverse radix");
  constexpr int LP = line_pitch(N);
  __shared__ Cx<float> tw[N];
  __shared__ Cx<float> xb[P * LP];  // exchanges, then the spectrum of f_z
  __shared__ Cx<float> sp[P * N];   // spectrum of f_x + i f_y
  const int tid = threadIdx.x;
  const int p = tid / TPL, t = tid % TPL;
  // a line's threads within one wavefront synchronise at wavefront scope; a line
  // that straddles wavefronts (TPL not dividing 64) uses block barriers
  constexpr bool WV = (64 % TPL == 0);
  const uint32_t line0 = (uint32_t)blockIdx.x * P;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  __syncthreads();  // the line transforms below synchronise only within a wavefront
  const LineView<float, 1> lv{xb + p * LP};
  const uint32_t lbase = (line0 + p) * (uint32_t)g.kzp;
  float fx[EPT], fy[EPT], fz[EPT];
  Cx<float> z[2][EPT];
  Cx<float> v[EPT];
  // raw half-spectrum pairs of the slices, loaded two slices ahead so that the
  // loads overlap the transforms (the barriers inside a transform keep the
  // compiler from moving later loads above it)
  Cx<float> ra[2][EPT], rb[2][EPT];
  auto fetch = [&](int q, Cx<float>* a, Cx<float>* b) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int pos = FI::in_at(t, i);
      const int k = pos <= HN ? pos : N - pos;
      a[i] = ld_masked(W + (2 * q) * g.wcomp, lbase + k, k < g.kzn);
      b[i] = ld_masked(W + (2 * q + 1) * g.wcomp, lbase + k, k < g.kzn);
    }
  };
  fetch(0, ra[0], rb[0]);
  fetch(1, ra[1], rb[1]);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int pos = FI::in_at(t, i);
      const Cx<float> a = ra[q & 1][i], bb = rb[q & 1][i];
      if (pos == 0 || pos == HN) v[i] = cx(a.re, bb.re);
      else if (pos < HN) v[i] = cx(a.re - bb.im, a.im + bb.re);
      else v[i] = cx(a.re + bb.im, bb.re - a.im);
    }
    if (q == 0) fetch(2, ra[0], rb[0]);
    FI::template run<WV>(v, t, lv, tw);
    if (q < 2) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) z[q][i] = v[i];
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const float ux = z[0][i].re, uy = z[0][i].im, uz = z[1][i].re, wx = z[1][i].im;
    const float wy = v[i].re, wz = v[i].im;
    fx[i] = uy * wz - uz * wy;
    fy[i] = uz * wx - ux * wz;
    fz[i] = ux * wy - uy * wx;
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) v[i] = cx(fx[i], fy[i]);
  FF::template run<WV>(v, t, lv, tw);
#pragma unroll
  for (int i = 0; i < EPT; ++i)
    if (FF::out_ok(t, i)) sp[p * N + FF::out_pos(t, i)] = v[i];
#pragma unroll
  for (int i = 0; i < EPT; ++i) v[i] = cx(fz[i], 0.f);
  FF::template run<WV>(v, t, lv, tw);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i)
    if (FF::out_ok(t, i)) xb[p * LP + FF::out_pos(t, i)] = v[i];
  __syncthreads();
  for (int idx = tid; idx < P * g.kzn; idx += NT) {
    const int k = idx % g.kzn, pp = idx / g.kzn;
    const Cx<float> c1 = sp[pp * N + k], c2 = sp[pp * N + ((N - k) % N)];
    const uint32_t off = (line0 + pp) * (uint32_t)g.kzp + k;
    st_off<stream_stores(N)>(W, off, cx(0.5f * (c1.re + c2.re), 0.5f * (c1.im - c2.im)));
    st_off<stream_stores(N)>(W + g.wcomp, off, cx(0.5f * (c1.im + c2.im), -0.5f * (c1.re - c2.re)));
    st_off<stream_stores(N)>(W + 2 * g.wcomp, off, xb[pp * LP + k]);
  }
}

// ------------------------------------------------------------------ x forward + epilogue
// FEED (0: none) names the stage output that is the next evaluation's input (1:
// out0, 2: out1).  The block then also runs that evaluation's x-inverse pass on
// its own tile (shift sh2): the values just computed are still in registers, at
// the input positions of the inverse transform (its first radix is the forward
// transform's last), so the tile is not read back.  An out1 that only feeds the
// next evaluation is not stored.  FEED needs a.full == 0 (the blocks are then the
// active tiles, the same as the x-inverse pass); CURL as in f_xinv.
template <typename C, int OP, int FEED, bool CURL>
__global__ void __launch_bounds__(kFastL * C::TPL)
f_xfwd(Cx<float>* __restrict__ W, const Cx<float>* __restrict__ twg, Shift sh, Shift sh2,
       const int2* __restrict__ tiles, Geom g, EpiArgs<float> a) {
  constexpr int N = C::N, TPL = C::TPL, EPT = C::EPT;
  using F = RegFft<N, TPL, -1, typename C::Fwd>;
  using FI = RegFft<N, TPL, +1, typename C::Inv>;
  static_assert(FEED == 0 || F::RL == FI::R0, "the inverse transform must start with the forward's last radix");
  __shared__ Cx<float> tw[N];
  __shared__ Cx<float> phx[N];
  __shared__ Cx<float> phc[kFastL];
  __shared__ Cx<float> phx2[FEED ? N : 1];
  __shared__ Cx<float> phc2[FEED ? kFastL : 1];
  __shared__ Cx<float> xb[N * kFastLp];
  const int tid = threadIdx.x;
  const int l = tid % kFastL, t = tid / kFastL;
  int yi, kz0;
  if (a.full) {
    yi = blockIdx.x / a.ntzf;
    kz0 = (blockIdx.x % a.ntzf) * kFastL;
  } else {
    const int2 tile = tiles[blockIdx.x];
    yi = tile.x;
    kz0 = tile.y;
  }
  const int kz = kz0 + l;
  const int ky = kval(yi, N);
  const bool active = line_active(g, ky, kz0);
  const LineView<float, kFastLp> lv{xb + l};
  Cx<float> r[3][EPT];
  Cx<float> phyz = cx(1.f, 0.f);
  // stage operands, read per chunk of points before that chunk's stores (out0 may
  // alias an operand, which keeps the compiler from hoisting loads above stores):
  // half of the points per chunk for two-operand stages, and for one-operand
  // stages at N <= 128 (fewer registers, four waves per SIMD instead of three;
  // measured faster there, slower at N = 256); the first chunk is read before the
  // last transform so that its latency overlaps it
  constexpr bool need0 = (OP == OP_HEUN1 || OP == OP_EX1B || OP == OP_EX2B || OP == OP_RK4_0 ||
                          OP == OP_RK4_1 || OP == OP_RK4_2 || OP == OP_MID1 || OP == OP_MID2 ||
                          OP == OP_EUL || OP == OP_EULAV);
  constexpr bool need1 = (OP == OP_AVG || OP == OP_HEUN2 || OP == OP_EX1B || OP == OP_EX2B ||
                          OP == OP_RK4_1 || OP == OP_RK4_2 || OP == OP_RK4_3 || OP == OP_ACC ||
                          OP == OP_EULAV);
  constexpr bool use1 = (OP == OP_HEUN1 || OP == OP_RK4_0 || OP == OP_RK4_1 || OP == OP_RK4_2) && FEED != 2;
  static_assert(FEED == 0 || op_can_feed(OP, FEED), "this stage output is not an evaluation input");
  Cx<float> nx[FEED ? 3 : 1][FEED ? EPT : 1];  // the fed output on this thread's points
  if constexpr (FEED != 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i = 0; i < EPT; ++i) nx[c][i] = cx(0.f, 0.f);
  }
  constexpr int CH = ((need0 && need1) || ((need0 || need1) && N <= 128)) ? (EPT + 1) / 2 : EPT;
  const LineTest keep = line_test(g, ky, kz);
  const bool line_kept = active && kz < g.kzn;
  // streaming stores into the compact stage buffers only (rows of whole 128-byte lines)
  const bool st0 = stream_stores(N) && a.lo0.pitch == g.kzp;
  [[maybe_unused]] const bool st1 = stream_stores(N) && a.lo1.pitch == g.kzp;
  Cx<float> s0v[need0 ? 3 : 1][need0 ? CH : 1], s1v[need1 ? 3 : 1][need1 ? CH : 1];
  auto load_ops = [&](int c0) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (c0 + j >= EPT) break;  // an odd register count: the second chunk is one short
      const int p = F::out_at(t, c0 + j);
      const bool ok = line_kept && F::out_ok(t, c0 + j) && keep(kval(p, N));
      if constexpr (need0) {
        const uint32_t ii0 = (uint32_t)((p * N + yi) * a.li0.pitch + kz);
#pragma unroll
        for (int c = 0; c < 3; ++c) s0v[c][j] = ld_masked(a.in0 + c * a.li0.cs, ii0, ok);
      }
      if constexpr (need1) {
        const uint32_t ii1 = (uint32_t)((p * N + yi) * a.li1.pitch + kz);
#pragma unroll
        for (int c = 0; c < 3; ++c) s1v[c][j] = ld_masked(a.in1 + c * a.li1.cs, ii1, ok);
      }
    }
  };
  if (active) {
    for (int i = tid; i < N; i += kFastL * TPL) tw[i] = twg[i];
    if (sh.on) {
      phase_row(phx, N, sh.s[0], tid, kFastL * TPL);
      phase_cols(phc, ky, kz0, sh, N, tid);
    }
    if constexpr (FEED != 0) {
      if (sh2.on) {
        phase_row(phx2, N, sh2.s[0], tid, kFastL * TPL);
        phase_cols(phc2, ky, kz0, sh2, N, tid);
      }
    }
    const bool col = kz < g.kzn;
    const uint32_t wbase = (uint32_t)(yi * g.kzp + kz0) + l, wstep = (uint32_t)(N * g.kzp);
    // field f + 1 is loaded while field f is transformed
#pragma unroll
    for (int i = 0; i < EPT; ++i) r[0][i] = ld_masked(W, (uint32_t)F::in_at(t, i) * wstep + wbase, col && F::in_ok(t, i));
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      if (f < 2) {
#pragma unroll
        for (int i = 0; i < EPT; ++i)
          r[f + 1][i] = ld_masked(W + (f + 1) * g.wcomp, (uint32_t)F::in_at(t, i) * wstep + wbase, col && F::in_ok(t, i));
      } else {
        load_ops(0);
      }
      F::run(r[f], t, lv, tw);  // its barriers also publish phx and phc
    }
    if (sh.on) phyz = phc[l];
  }
  const bool epi_on = !(kz >= g.h || (!a.full && kz >= g.kzn));
  if (FEED == 0 && !epi_on) return;
  const float inv_n3 = 1.f / (float(N) * float(N) * float(N));
  if (epi_on) {
#pragma unroll
  for (int c0 = 0; c0 < EPT; c0 += CH) {
  if (c0 > 0 || !active) load_ops(c0);
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const int i = c0 + j;
    if (i >= EPT) break;
    if (!F::out_ok(t, i)) continue;  // no point in this register
    const int p = F::out_pos(t, i);
    const int kx = kval(p, N);
    const uint32_t io0 = (uint32_t)((p * N + yi) * a.lo0.pitch + kz);
    if (!(line_kept && keep(kx))) {
      // outside the retained set: zero in outputs that must be complete (full
      // mode, the caller's arrays); stage buffers are only read at retained modes
      if (a.full)
        for (int c = 0; c < 3; ++c) st_off(a.out0 + c * a.lo0.cs, io0, cx(0.f, 0.f));
      continue;
    }
    const uint32_t io1 = use1 ? (uint32_t)((p * N + yi) * a.lo1.pitch + kz) : 0u;
    Cx<float> Fv[3] = {scale(r[0][i], inv_n3), scale(r[1][i], inv_n3), scale(r[2][i], inv_n3)};
    if (sh.on) {
      const Cx<float> phi = cmul(phx[p], phyz);
      Fv[0] = cmulc(Fv[0], phi);
      Fv[1] = cmulc(Fv[1], phi);
      Fv[2] = cmulc(Fv[2], phi);
    }
    const int k2 = kx * kx + ky * ky + kz * kz;
    if (k2 == 0) {
      Fv[0] = Fv[1] = Fv[2] = cx(0.f, 0.f);
    } else {
      const float rk2 = 1.f / float(k2);
      const float kxr = float(kx), kyr = float(ky), kzr = float(kz);
      const Cx<float> kd = scale(scale(Fv[0], kxr) + scale(Fv[1], kyr) + scale(Fv[2], kzr), rk2);
      Fv[0] = Fv[0] - scale(kd, kxr);
      Fv[1] = Fv[1] - scale(kd, kyr);
      Fv[2] = Fv[2] - scale(kd, kzr);
    }
    float eh = 1.f, edt = 1.f;
    if (op_uses_etab(OP)) { eh = a.eh[k2]; edt = a.edt[k2]; }
    const float dt = a.dt;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Cx<float>* out0 = a.out0 + c * a.lo0.cs;
      Cx<float>* out1 = use1 ? a.out1 + c * a.lo1.cs : nullptr;
      Cx<float> Nv = Fv[c];
      Cx<float> O = cx(0.f, 0.f);
      if (op_forced(OP) && a.force != nullptr && k2 >= 4 && k2 <= 9)
        O = a.force[c * 196 + ((kx + 3) * 7 + (ky + 3)) * 4 + kz];
      if (OP != OP_HEUN1) Nv = Nv + O;  // RK4 slopes N + O (zero for the other ops)
      Cx<float> s0 = cx(0.f, 0.f), s1 = cx(0.f, 0.f);
      if constexpr (need0) s0 = s0v[c][j];
      if constexpr (need1) s1 = s1v[c][j];
      Cx<float> v0 = cx(0.f, 0.f), v1 = cx(0.f, 0.f);
      if (OP == OP_STORE) {
        v0 = Nv;
      } else if (OP == OP_AVG) {
        v0 = scale(s1 + Nv, 0.5f);
      } else if (OP == OP_HEUN1) {
        v1 = scale(s0 + scale(Nv + O, dt), edt);
        v0 = scale(s0, edt) + scale(Nv + O + O, 0.5f * dt * eh);
      } else if (OP == OP_HEUN2) {
        v0 = s1 + scale(Nv, 0.5f * dt * eh);
      } else if (OP == OP_EX1B) {
        v0 = scale(s0 + scale(s1 + Nv, 0.5f * dt * a.w), eh);
      } else if (OP == OP_EX2B) {
        v0 = scale(s0, edt) + scale(s1 + Nv, dt * a.w * eh);
      } else if (OP == OP_RK4_0) {
        v1 = scale(s0 + scale(Nv, 0.5f * dt), eh);
        v0 = scale(s0 + scale(Nv, dt / 6.f), edt);
      } else if (OP == OP_RK4_1) {
        v1 = scale(s0, eh) + scale(Nv, 0.5f * dt);
        v0 = s1 + scale(Nv, dt / 3.f * eh);
      } else if (OP == OP_RK4_2) {
        v1 = scale(s0, edt) + scale(Nv, dt * eh);
        v0 = s1 + scale(Nv, dt / 3.f * eh);
      } else if (OP == OP_RK4_3) {
        v0 = s1 + scale(Nv, dt / 6.f);
      } else if (OP == OP_ACC) {
        v0 = s1 + Nv;
      } else if (OP == OP_MID1) {
        v0 = scale(s0 + scale(Nv, 0.5f * dt), eh);
      } else if (OP == OP_MID2) {
        v0 = scale(s0, edt) + scale(Nv, dt * eh);
      } else if (OP == OP_EUL) {
        v0 = scale(s0 + scale(Nv, dt), edt);
      } else {  // OP_EULAV
        v0 = scale(s0 + scale(s1 + Nv, dt * a.w), edt);
      }
      if constexpr (use1) {
        if (st1) st_off<true>(out1, io1, v1);
        else st_off(out1, io1, v1);
      }
      if (st0) st_off<true>(out0, io0, v0);
      else st_off(out0, io0, v0);
      if constexpr (FEED == 1) nx[c][i] = v0;
      if constexpr (FEED == 2) nx[c][i] = v1;
    }
  }
  }
  }
  if constexpr (FEED != 0) {
    // the next evaluation's x-inverse pass on this tile (as f_xinv<C, CURL>, from registers)
    const bool col = kz < g.kzn;
    Cx<float> ux[EPT], uy[EPT], uz[EPT], dy[EPT], dz[EPT];
    [[maybe_unused]] const float kyf = float(ky), kzf = float(kz);
    const Cx<float> phyz2 = sh2.on ? phc2[l] : cx(1.f, 0.f);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int p = FI::in_at(t, i);
      ux[i] = nx[0][i];
      uy[i] = nx[1][i];
      uz[i] = nx[2][i];
      if (sh2.on) {
        const Cx<float> phi = cmul(phx2[p], phyz2);
        ux[i] = cmul(ux[i], phi);
        uy[i] = cmul(uy[i], phi);
        uz[i] = cmul(uz[i], phi);
      }
      const float kxf = float(kval(p, N));
      dy[i] = mul_i(scale(uy[i], kxf));
      dz[i] = mul_i(scale(uz[i], kxf));
    }
    const uint32_t obase = (uint32_t)(yi * g.kzp + kz0) + l, ostep = (uint32_t)(N * g.kzp);
    auto store = [&](int f, const Cx<float>* v) {
      if (col) {
#pragma unroll
        for (int i = 0; i < EPT; ++i)
          if (FI::out_ok(t, i))
            st_off<stream_stores(N)>(W + f * g.wcomp, (uint32_t)FI::out_pos(t, i) * ostep + obase, v[i]);
      }
    };
    FI::run(uy, t, lv, tw);
    store(1, uy);
    FI::run(uz, t, lv, tw);
    store(2, uz);
    if constexpr (CURL) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) uy[i] = mul_i(scale(uz[i], kyf) - scale(uy[i], kzf));  // omega_x
      store(3, uy);
    }
    FI::run(ux, t, lv, tw);
    store(0, ux);
    FI::run(dz, t, lv, tw);
    if constexpr (CURL) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) dz[i] = mul_i(scale(ux[i], kzf)) - dz[i];  // omega_y
    }
    store(4, dz);
    FI::run(dy, t, lv, tw);
    if constexpr (CURL) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) dy[i] = dy[i] - mul_i(scale(ux[i], kyf));  // omega_z
    }
    store(5, dy);
  }
}

// Specialised sizes (FP32).  The forward radix list is the inverse one reversed.
// YC (the vorticity formed in the y-inverse pass, f_ycurl) is on for 128, 144, 256
// and 270, where the x-inverse passes writing five fields instead of six gain more
// than the y-inverse pass loses to its three-field blocks: PS-RK2 random steps
// 3.3%, 1.3%, 2.8% and 1.5% faster.  At 64, 160, 192, 216, 324, 360, 384 and 512
// those blocks leave one or two resident a CU and the step was 0.3% to 13% slower;
// 240 was unchanged.
using LP64 = LinePlan<64, 8, Radices<8, 8>, Radices<8, 8>>;
using LP128b = LinePlan<128, 16, Radices<8, 4, 4>, Radices<4, 4, 8>>;
using LP192 = LinePlan<192, 16, Radices<12, 4, 4>, Radices<4, 4, 12>>;
using LP256b = LinePlan<256, 32, Radices<8, 8, 4>, Radices<4, 8, 8>>;
using Fast64 = FastCfg<LP64, LP64, LP64, 16, LP64>;
using Fast128 = FastCfg<LP128b, LP128b, LP128b, 8, LP128b, LP128b, 8, true>;
// z pass of 192: 6 8 4 over 32 threads, 8 registers a transform (the adjoint z
// pass keeps 12 4 4 over 16)
using LP192z = LinePlan<192, 32, Radices<6, 8, 4>, Radices<4, 8, 6>>;
using Fast192 = FastCfg<LP192, LP192, LP192z, 8, LP192, LP192, 8>;
// z pass of 256: 4 4 4 4 over 64 threads (4 registers a transform, six waves per
// SIMD; 5% faster than 8 8 4 over 32 at 256^3, whose extra exchange costs more at
// 128^3); the adjoint z pass keeps 8 8 4 over 32
using LP256z = LinePlan<256, 64, Radices<4, 4, 4, 4>, Radices<4, 4, 4, 4>>;
using Fast256 = FastCfg<LP256b, LP256b, LP256z, 4, LP256b, LP256b, 8, true>;
// 216 = 12 6 3 and 324 = 12 3 3 3 with 12 points per thread (18 and 27 threads per
// line): the grids of the k_max = 108 comparison
using LP216 = LinePlan<216, 18, Radices<12, 6, 3>, Radices<3, 6, 12>>;
using LP324 = LinePlan<324, 27, Radices<12, 3, 3, 3>, Radices<3, 3, 3, 12>>;
// z passes with the line inside one wavefront (wavefront-scope synchronisation
// instead of block barriers) and few registers a thread (more waves per SIMD),
// some butterflies predicated off: 216 = 8 3 9 over 32 threads (9 registers),
// 324 = 6 6 9 over 64 (9); the adjoint z pass of 324 keeps 12 3 3 3 over 32
using LP216z = LinePlan<216, 32, Radices<8, 3, 9>, Radices<9, 3, 8>>;
using LP324z = LinePlan<324, 64, Radices<6, 6, 9>, Radices<9, 6, 6>>;
using LP324za = LinePlan<324, 32, Radices<12, 3, 3, 3>, Radices<3, 3, 3, 12>>;
// 216 and 240 run their x passes on the z plans too (32 threads a line, 512-thread
// tiles of 8 waves, 156-161 registers a thread) rather than on 18 and 24 threads a
// line (5 and 6 waves a tile, one tile per CU): fused x pass 152 -> 132 us at 216^3,
// 154 -> 146 us at 240^3
using Fast216 = FastCfg<LP216z, LP216, LP216z, 4, LP216z>;
using Fast324 = FastCfg<LP324, LP324, LP324z, 4, LP324, LP324za, 4>;
// 384 = 12 4 4 2 (inverse), 32 threads per line, four lines per z block
using LP384 = LinePlan<384, 32, Radices<12, 4, 4, 2>, Radices<2, 4, 4, 12>>;
// z pass of 384: 6 8 8 over 64 threads, 8 registers and two exchanges a transform
// (the adjoint z pass keeps 12 4 4 2 over 32)
using LP384z = LinePlan<384, 64, Radices<6, 8, 8>, Radices<8, 8, 6>>;
using Fast384 = FastCfg<LP384, LP384, LP384z, 4, LP384, LP384, 4>;
// 512 (the 2/3-truncated RK4 grid of the 512^3 comparison): y and z passes 8 8 8
// with one wavefront per line, four lines per z block (at eight, one 512-thread
// block of about 130 registers a thread is all a CU holds); x passes 16 8 4 with
// 32 threads per line, so that a 16-column tile is a 512-thread block of up to 256
// registers a thread (the chained x pass still spills some, but fewer waves per
// line and more registers measured faster than 1024-thread tiles of 128)
using LP512 = LinePlan<512, 64, Radices<8, 8, 8>, Radices<8, 8, 8>>;
using LP512x = LinePlan<512, 32, Radices<16, 8, 4>, Radices<4, 8, 16>>;
using Fast512 = FastCfg<LP512x, LP512, LP512, 4, LP512x>;
// Grids whose radices do not all divide one points-per-thread count: 12 registers
// a thread, some butterflies of a stage predicated off (fft_reg.hpp).  144 = 12 12
// (uniform, 12 threads), 160 = 10 4 4 (16), 240 = 10 4 6 (24), 270 = 9 6 5 (30),
// 360 = 10 6 6 (36, the y pass): the truncation sweeps at k_max = 64 and 108 and the
// coarse grid of the 512^3 comparison at C_t = 0.948.
using LP144 = LinePlan<144, 12, Radices<12, 12>, Radices<12, 12>>;
using LP160 = LinePlan<160, 16, Radices<10, 4, 4>, Radices<4, 4, 10>>;
using LP240 = LinePlan<240, 24, Radices<10, 4, 6>, Radices<6, 4, 10>>;
using LP270 = LinePlan<270, 30, Radices<9, 6, 5>, Radices<5, 6, 9>>;
using LP360 = LinePlan<360, 36, Radices<10, 6, 6>, Radices<6, 6, 10>>;
// x passes of 360: 30 threads per line (12 6 5, up to 15 registers a transform), so
// that a 16-column tile is a 480-thread block that may hold 256 registers a thread
// (576 threads allow 168, and the x-forward passes spilled)
using LP360x = LinePlan<360, 30, Radices<12, 6, 5>, Radices<5, 6, 12>>;
// z passes with lines inside one wavefront and few registers a thread: 144 = 6 6 4,
// 160 = 4 8 5, 240 = 8 6 5, 270 = 10 3 9, 360 = 12 6 5, all over 32 threads (8 to
// 15 registers a transform); the adjoint z passes of 160 and 360, which hold eight
// slices, keep 10 4 4 over 16 and 10 6 6 over 64
using LP144z = LinePlan<144, 32, Radices<6, 6, 4>, Radices<4, 6, 6>>;
using LP240z = LinePlan<240, 32, Radices<8, 6, 5>, Radices<5, 6, 8>>;
using LP270z = LinePlan<270, 32, Radices<10, 3, 9>, Radices<9, 3, 10>>;
using LP360z = LinePlan<360, 32, Radices<12, 6, 5>, Radices<5, 6, 12>>;
using LP360za = LinePlan<360, 64, Radices<10, 6, 6>, Radices<6, 6, 10>>;
using Fast144 = FastCfg<LP144, LP144, LP144z, 8, LP144, LP144z, 8, true>;
using LP160z = LinePlan<160, 32, Radices<4, 8, 5>, Radices<5, 8, 4>>;
using Fast160 = FastCfg<LP160, LP160, LP160z, 8, LP160, LP160, 8>;
using Fast240 = FastCfg<LP240z, LP240, LP240z, 4, LP240z>;
using Fast270 = FastCfg<LP270, LP270, LP270z, 4, LP270, LP270z, 4, true>;
using Fast360 = FastCfg<LP360x, LP360, LP360z, 4, LP360x, LP360za, 4>;

}  // namespace ns
