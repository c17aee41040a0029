// ns_kernels.hpp -- HIP kernels (gfx950) of one evaluation of the dealiased
// nonlinear term N(u) = M conj(phi) P FFT( IFFT(phi u) x IFFT(i k x phi u) ) and of
// the integrating-factor Runge-Kutta stage updates fused behind it.
//
// Five launches per evaluation, all bandwidth-bound:
//   k_xinv   state -> scratch: phase shift, curl, inverse FFT along x (6 fields);
//            the shift factors are generated per block in FP64 and rounded once
//   k_ypass  scratch in place: inverse FFT along y (6 fields)
//   k_zcross scratch in place: c2r along z (6 fields), u x omega, r2c along z (3 fields)
//   k_ypass  scratch in place: forward FFT along y (3 fields)
//   k_xfwd   scratch -> state: forward FFT along x, 1/N^3, deshift, projection,
//            truncation mask, and the Runge-Kutta stage combination
// Scratch layout: field f, [x or k_x][y or k_y][k_z < kzn], k_z stride kzp.
// Only the k_z planes and (k_y, k_z) lines that can hold retained modes are
// transformed; everything else is known to be zero and is neither read nor
// written (a pruned transform: the truncation sphere or cube bounds the support).
#pragma once

#include "fft_core.hpp"

namespace ns {

struct Geom {
  int n, h;         // N, N/2 + 1
  int kzn;          // k_z planes that can hold retained modes (k_z < kzn)
  int kzp;          // k_z stride of the scratch fields (kzn rounded up)
  int L;            // k_z columns per strided tile (power of two)
  int lgL;          // log2(L)
  int mask;         // 0 sphere, 1 cube, 2 sphere / 3 cube without the double-alias reach
  int kmax;         // largest retained |k_i|
  long long k2max;  // sphere: largest retained |k|^2; cube: 3 kmax^2
  long long comp;   // state component stride, n*n*h
  long long wcomp;  // scratch field stride, n*n*kzp
};

__device__ __forceinline__ int kval(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// |k_i| + |k_j| < 2N/3 for every pair of axes: a state held in this set never
// receives a double alias (a pair sum reaching k + N(s_i e_i + s_j e_j) would need
// |q_i| + |q_j| >= 2N - |k_i| - |k_j| > 4N/3, more than two such modes can add up to).
__device__ __forceinline__ bool double_alias_free(const Geom& g, int kx, int ky, int kz) {
  const int a = abs(kx), b = abs(ky), c = abs(kz), n2 = 2 * g.n;
  return 3 * (a + b) < n2 && 3 * (a + c) < n2 && 3 * (b + c) < n2;
}

__device__ __forceinline__ bool cube_family(const Geom& g) { return g.mask == 1 || g.mask == 3; }

__device__ __forceinline__ bool retained(const Geom& g, int kx, int ky, int kz) {
  if (cube_family(g)) {
    if (abs(kx) > g.kmax || abs(ky) > g.kmax || kz > g.kmax) return false;
  } else if ((long long)kx * kx + (long long)ky * ky + (long long)kz * kz > g.k2max) {
    return false;
  }
  return g.mask < 2 || double_alias_free(g, kx, ky, kz);
}

__device__ __forceinline__ int isqrt_ll(long long v) {
  if (v < 0) return -1;
  int r = (int)sqrt((double)v);
  while ((long long)r * r > v) --r;
  while ((long long)(r + 1) * (r + 1) <= v) ++r;
  return r;
}

// Largest |k_y| that can be retained on k_z plane kz (-1: none); for the masks
// without the double-alias reach the bound of their sphere or cube (a superset).
__device__ __forceinline__ int ybound(const Geom& g, int kz) {
  if (!cube_family(g)) return isqrt_ll(g.k2max - (long long)kz * kz);
  return kz <= g.kmax ? g.kmax : -1;
}

__device__ __forceinline__ bool line_active(const Geom& g, int ky, int kz) {
  return kz < g.kzn && abs(ky) <= ybound(g, kz);
}

template <typename R>
__device__ __forceinline__ Cx<R> mul_i(Cx<R> a) { return cx(-a.im, a.re); }

// Addressing of a state-shaped array: the caller's layout [3][N][N][N/2+1]
// (pitch N/2+1) or the compact internal one [3][N][N][kzp] (k_z < kzn only,
// rows aligned to the tile width).
struct Lay {
  int pitch;        // k_z pitch of a (k_x, k_y) row
  long long cs;     // component stride
};
__device__ __forceinline__ long long lay_at(const Lay& L, int xi, int yi, int kz, int n) {
  return ((long long)xi * n + yi) * L.pitch + kz;
}

// Grid shift s (grid-spacing units); on == 0: unshifted.
struct Shift {
  double s[3];
  int on;
};
// exp(2 pi i k s / N), evaluated in FP64 (sincospi) and rounded once.
template <typename R>
__device__ __forceinline__ Cx<R> phase1(int k, double s, int n) {
  double sn, cs;
  sincospi(2.0 * (double)k * s / (double)n, &sn, &cs);
  return cx(R(cs), R(sn));
}
// Per-block table of the k_x factors: ph[i] = exp(2 pi i kval(i) s_x / N).
template <typename R>
__device__ __forceinline__ void phase_row(Cx<R>* ph, int n, double s, int tid, int nt) {
  for (int i = tid; i < n; i += nt) ph[i] = phase1<R>(kval(i, n), s, n);
}

// ------------------------------------------------------------------ k_xinv
// One block per active (k_y, k_z tile); points p = k_x index, columns l = k_z - kz0.
// Holds the three velocity components in registers and sends the six fields
// u_x, u_y, u_z, omega_x, omega_y, omega_z one after the other through LDS.
template <typename R, int EPT>
__global__ void __launch_bounds__(512)
k_xinv(const Cx<R>* __restrict__ S, Lay ls, Cx<R>* __restrict__ W, const Cx<R>* __restrict__ twg,
       Shift sh, const int2* __restrict__ tiles, Geom g, FftPlan plan) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem_raw);
  Cx<R>* phx = tw + g.n;
  Cx<R>* buf = phx + g.n;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = g.n, L = g.L;
  const int2 tile = tiles[blockIdx.x];
  const int yi = tile.x, kz0 = tile.y;
  const int ky = kval(yi, n);
  const int npts = n * L;
  for (int t = tid; t < n; t += nt) tw[t] = twg[t];
  if (sh.on) phase_row(phx, n, sh.s[0], tid, nt);
  __syncthreads();
  const Cx<R> phy = sh.on ? phase1<R>(ky, sh.s[1], n) : cx(R(1), R(0));

  Cx<R> u[3][EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nt;
    u[0][i] = u[1][i] = u[2][i] = cx(R(0), R(0));
    if (e < npts) {
      const int p = e >> g.lgL, l = e & (L - 1);
      const int kz = kz0 + l, kx = kval(p, n);
      if (kz < g.kzn && retained(g, kx, ky, kz)) {
        const long long idx = lay_at(ls, p, yi, kz, n);
        u[0][i] = S[idx];
        u[1][i] = S[ls.cs + idx];
        u[2][i] = S[2 * ls.cs + idx];
        if (sh.on) {
          const Cx<R> phi = cmul(phx[p], cmul(phy, phase1<R>(kz, sh.s[2], n)));
          u[0][i] = cmul(u[0][i], phi);
          u[1][i] = cmul(u[1][i], phi);
          u[2][i] = cmul(u[2][i], phi);
        }
      }
    }
  }
  for (int f = 0; f < 6; ++f) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nt;
      if (e < npts) {
        const int p = e >> g.lgL, l = e & (L - 1);
        const R kx = R(kval(p, n)), kyr = R(ky), kz = R(kz0 + l);
        Cx<R> v;
        switch (f) {
          case 0: v = u[0][i]; break;
          case 1: v = u[1][i]; break;
          case 2: v = u[2][i]; break;
          case 3: v = mul_i(scale(u[2][i], kyr) - scale(u[1][i], kz)); break;
          case 4: v = mul_i(scale(u[0][i], kz) - scale(u[2][i], kx)); break;
          default: v = mul_i(scale(u[1][i], kx) - scale(u[0][i], kyr)); break;
        }
        buf[e] = v;
      }
    }
    __syncthreads();
    fft_lines<+1, EPT, true>(buf, tw, plan, L, L, 1, tid, nt);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nt;
      if (e < npts) {
        const int p = e >> g.lgL, l = e & (L - 1);
        const int kz = kz0 + l;
        if (kz < g.kzn) W[f * g.wcomp + ((long long)p * n + yi) * g.kzp + kz] = buf[e];
      }
    }
  }
}

// ------------------------------------------------------------------ k_ypass
// Blocks over (field, x, k_z tile); in place.  S = +1 inverse (reads only the
// k_y rows that can be non-zero), S = -1 forward (writes only those rows).
template <typename R, int EPT, int S>
__global__ void __launch_bounds__(512)
k_ypass(Cx<R>* __restrict__ W, const Cx<R>* __restrict__ twg, int f0, int ntz, Geom g,
        FftPlan plan) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem_raw);
  Cx<R>* buf = tw + g.n;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = g.n, L = g.L;
  const int b = blockIdx.x;
  const int kzt = b % ntz;
  const int rest = b / ntz;
  const int x = rest % n;
  const int f = f0 + rest / n;
  const int kz0 = kzt * L;
  const int yb = ybound(g, kz0);
  const int npts = n * L;
  Cx<R>* base = W + f * g.wcomp + (long long)x * n * g.kzp;
  for (int t = tid; t < n; t += nt) tw[t] = twg[t];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nt;
    if (e < npts) {
      const int p = e >> g.lgL, l = e & (L - 1);
      const int kz = kz0 + l;
      Cx<R> v = cx(R(0), R(0));
      if (kz < g.kzn && (S < 0 || abs(kval(p, n)) <= yb)) v = base[(long long)p * g.kzp + kz];
      buf[e] = v;
    }
  }
  __syncthreads();
  fft_lines<S, EPT, true>(buf, tw, plan, L, L, 1, tid, nt);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nt;
    if (e < npts) {
      const int p = e >> g.lgL, l = e & (L - 1);
      const int kz = kz0 + l;
      if (kz < g.kzn && (S > 0 || abs(kval(p, n)) <= yb)) base[(long long)p * g.kzp + kz] = buf[e];
    }
  }
}

// ------------------------------------------------------------------ k_zcross
// P (even) consecutive (x, y) lines per block.  Two real lines a, b are carried
// by one complex line z = a + i b: from the half spectra, Z(k) = a(k) + i b(k)
// and Z(N-k) = conj(a(k)) + i conj(b(k)); after the forward transform,
// a(k) = (Z(k) + conj Z(N-k))/2 and b(k) = (Z(k) - conj Z(N-k))/(2i).  As a c2r
// transform does, the imaginary parts of the k_z = 0 coefficients are dropped.
// Inverse pairs: (u_x, u_y), (u_z, w_x), (w_y, w_z); forward pairs: (f_x, f_y)
// of each line and f_z of lines 2j, 2j+1.  Output is unnormalised.
template <typename R, int EPT>
__global__ void __launch_bounds__(512)
k_zcross(Cx<R>* __restrict__ W, const Cx<R>* __restrict__ twg, int P, Geom g, FftPlan plan) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem_raw);
  Cx<R>* buf = tw + g.n;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = g.n, hn = n / 2;
  const long long line0 = (long long)blockIdx.x * P;
  for (int t = tid; t < n; t += nt) tw[t] = twg[t];
  // load: (line p, pair q, k in [0, N/2])
  const int nk = hn + 1;
  for (int idx = tid; idx < P * 3 * nk; idx += nt) {
    const int k = idx % nk;
    const int rest = idx / nk;
    const int q = rest % 3, p = rest / 3;
    Cx<R> a = cx(R(0), R(0)), bb = cx(R(0), R(0));
    if (k < g.kzn) {
      const long long off = (line0 + p) * g.kzp + k;
      a = W[(2 * q) * g.wcomp + off];
      bb = W[(2 * q + 1) * g.wcomp + off];
    }
    Cx<R>* z = buf + (p * 3 + q) * n;
    if (k == 0 || k == hn) {
      z[k] = cx(a.re, bb.re);
    } else {
      z[k] = cx(a.re - bb.im, a.im + bb.re);
      z[n - k] = cx(a.re + bb.im, bb.re - a.im);
    }
  }
  __syncthreads();
  fft_lines<+1, EPT, false>(buf, tw, plan, 3 * P, 1, n, tid, nt);
  // product u x omega at every point; results buffered in registers, then written
  // to forward lines: slot p = f_x + i f_y of line p, slot P + j = f_z(2j) + i f_z(2j+1)
  constexpr int PPT = (EPT + 2) / 3;  // points per thread: P*n <= EPT*nt/3
  R fx[PPT], fy[PPT], fz[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int e = tid + i * nt;
    if (e < P * n) {
      const int p = e / n, j = e % n;
      const Cx<R> z0 = buf[(p * 3) * n + j], z1 = buf[(p * 3 + 1) * n + j], z2 = buf[(p * 3 + 2) * n + j];
      const R ux = z0.re, uy = z0.im, uz = z1.re, wx = z1.im, wy = z2.re, wz = z2.im;
      fx[i] = uy * wz - uz * wy;
      fy[i] = uz * wx - ux * wz;
      fz[i] = ux * wy - uy * wx;
    }
  }
  __syncthreads();
  R* bufr = reinterpret_cast<R*>(buf);
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int e = tid + i * nt;
    if (e < P * n) {
      const int p = e / n, j = e % n;
      buf[p * n + j] = cx(fx[i], fy[i]);
      bufr[2 * ((P + p / 2) * n + j) + (p & 1)] = fz[i];
    }
  }
  __syncthreads();
  fft_lines<-1, EPT, false>(buf, tw, plan, P + P / 2, 1, n, tid, nt);
  // unpack the k_z < kzn coefficients of the three real fields
  for (int idx = tid; idx < (P + P / 2) * g.kzn; idx += nt) {
    const int k = idx % g.kzn, s = idx / g.kzn;
    const Cx<R> c1 = buf[s * n + k];
    const Cx<R> c2 = buf[s * n + ((n - k) % n)];
    const Cx<R> a = cx(R(0.5) * (c1.re + c2.re), R(0.5) * (c1.im - c2.im));
    const Cx<R> bb = cx(R(0.5) * (c1.im + c2.im), R(-0.5) * (c1.re - c2.re));
    if (s < P) {
      const long long off = (line0 + s) * g.kzp + k;
      W[off] = a;
      W[g.wcomp + off] = bb;
    } else {
      const int j = s - P;
      W[2 * g.wcomp + (line0 + 2 * j) * g.kzp + k] = a;
      W[2 * g.wcomp + (line0 + 2 * j + 1) * g.kzp + k] = bb;
    }
  }
}

// ------------------------------------------------------------------ k_xfwd
enum EpiOp {
  OP_STORE = 0,  // out0 = N
  OP_AVG = 1,    // out0 = (in1 + N)/2
  OP_HEUN1 = 2,  // out1 = E_dt (S0 + dt (N + O)); out0 = E_dt S0 + dt/2 E_h (N + 2 O)
  OP_HEUN2 = 3,  // out0 = in1 + dt/2 E_h N
  OP_EX1B = 4,   // out0 = E_h (S0 + dt/2 w (in1 + N))
  OP_EX2B = 5,   // out0 = E_dt S0 + dt E_h w (in1 + N)
  OP_RK4_0 = 6,  // out1 = E_h (S0 + dt/2 N); out0 = E_dt S0 + dt/6 E_dt N   (N: slope N + O)
  OP_RK4_1 = 7,  // out1 = E_h S0 + dt/2 N;   out0 = in1 + dt/3 E_h N
  OP_RK4_2 = 8,  // out1 = E_dt S0 + dt E_h N; out0 = in1 + dt/3 E_h N
  OP_RK4_3 = 9,  // out0 = in1 + dt/6 N
  OP_ACC = 10,   // out0 = in1 + N
  OP_MID1 = 11,  // out0 = E_h (S0 + dt/2 N)
  OP_MID2 = 12,  // out0 = E_dt S0 + dt E_h N
  OP_EUL = 13,   // out0 = E_dt (S0 + dt N)
  OP_EULAV = 14  // out0 = E_dt (S0 + dt w (in1 + N))
};
// w (EpiArgs::w) weighs each of the shifted evaluations summed in in1 + N: 1/2 for
// the two-shift average, 1/8 for the average over the eight shifts in {0, 1/2}^3.

// Ops that take the forcing O (EpiArgs::force, when non-null): the first Heun stage
// (which also carries the second stage's O into out0) and every RK4 stage, whose
// slope is N + O.
__host__ __device__ constexpr bool op_forced(int op) {
  return op == OP_HEUN1 || op == OP_RK4_0 || op == OP_RK4_1 || op == OP_RK4_2 || op == OP_RK4_3;
}

// Ops whose stage formula uses the integrating factors E_h and E_dt.
__host__ __device__ constexpr bool op_uses_etab(int op) {
  return op != OP_STORE && op != OP_AVG && op != OP_ACC;
}

// Stage outputs that are the next evaluation's input in the step sequences (feed
// 1: out0, 2: out1), for which the x-forward pass can also run that evaluation's
// x-inverse pass.
__host__ __device__ constexpr bool op_can_feed(int op, int feed) {
  return (feed == 2 && (op == OP_HEUN1 || op == OP_RK4_0 || op == OP_RK4_1 || op == OP_RK4_2)) ||
         (feed == 1 && (op == OP_HEUN2 || op == OP_RK4_3 || op == OP_EX1B || op == OP_EX2B));
}

template <typename R>
struct EpiArgs {
  Cx<R>* out0;
  Cx<R>* out1;
  const Cx<R>* in0;   // S0
  const Cx<R>* in1;   // accumulator; may alias out0
  Lay lo0, lo1, li0, li1;  // layouts of out0, out1, in0, in1
  const R* eh;        // exp(-nu k^2 dt/2) indexed by integer k^2
  const R* edt;       // exp(-nu k^2 dt)
  const Cx<R>* force; // [3][7][7][4] forcing on |k_i| <= 3, or null
  R dt;
  R w;                // weight of each summed evaluation (OP_EX1B, OP_EX2B, OP_EULAV)
  int full;           // 1: blocks cover every (k_y, k_z tile) of the half spectrum and write zeros outside
  int ntzf;           // k_z tiles over [0, N/2] in full mode
};

template <typename R, int EPT, int OP>
__global__ void __launch_bounds__(512)
k_xfwd(const Cx<R>* __restrict__ W, const Cx<R>* __restrict__ twg, Shift sh,
       const int2* __restrict__ tiles, Geom g, FftPlan plan, EpiArgs<R> a) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem_raw);
  Cx<R>* phx = tw + g.n;
  Cx<R>* buf = phx + g.n;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = g.n, L = g.L;
  int yi, kz0;
  if (a.full) {
    yi = blockIdx.x / a.ntzf;
    kz0 = (blockIdx.x % a.ntzf) * L;
  } else {
    const int2 tile = tiles[blockIdx.x];
    yi = tile.x;
    kz0 = tile.y;
  }
  const int ky = kval(yi, n);
  const bool active = line_active(g, ky, kz0);
  const int npts = n * L;
  Cx<R> r[3][EPT];
  if (active) {
    for (int t = tid; t < n; t += nt) tw[t] = twg[t];
    if (sh.on) phase_row(phx, n, sh.s[0], tid, nt);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      if (f > 0) __syncthreads();
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * nt;
        if (e < npts) {
          const int p = e >> g.lgL, l = e & (L - 1);
          const int kz = kz0 + l;
          Cx<R> v = cx(R(0), R(0));
          if (kz < g.kzn) v = W[f * g.wcomp + ((long long)p * n + yi) * g.kzp + kz];
          buf[e] = v;
        }
      }
      __syncthreads();
      fft_lines<-1, EPT, true>(buf, tw, plan, L, L, 1, tid, nt);
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * nt;
        r[f][i] = (e < npts) ? buf[e] : cx(R(0), R(0));
      }
    }
  }
  const R inv_n3 = R(1) / (R(n) * R(n) * R(n));
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nt;
    if (e >= npts) continue;
    const int p = e >> g.lgL, l = e & (L - 1);
    const int kz = kz0 + l;
    if (kz >= g.h || (!a.full && kz >= g.kzn)) continue;
    const int kx = kval(p, n);
    const long long io0 = lay_at(a.lo0, p, yi, kz, n);
    const bool ret = active && kz < g.kzn && retained(g, kx, ky, kz);
    if (!ret) {
      // zero outside the retained set only where the output must be complete (full
      // mode writes the caller's arrays, which carry no second output)
      if (a.full)
        for (int c = 0; c < 3; ++c) a.out0[c * a.lo0.cs + io0] = cx(R(0), R(0));
      continue;
    }
    const long long io1 = lay_at(a.lo1, p, yi, kz, n);
    const long long ii0 = lay_at(a.li0, p, yi, kz, n);
    const long long ii1 = lay_at(a.li1, p, yi, kz, n);
    Cx<R> F[3] = {scale(r[0][i], inv_n3), scale(r[1][i], inv_n3), scale(r[2][i], inv_n3)};
    if (sh.on) {
      const Cx<R> phi = cmul(cmul(phx[p], phase1<R>(ky, sh.s[1], n)), phase1<R>(kz, sh.s[2], n));
      F[0] = cmulc(F[0], phi);
      F[1] = cmulc(F[1], phi);
      F[2] = cmulc(F[2], phi);
    }
    const long long k2 = (long long)kx * kx + (long long)ky * ky + (long long)kz * kz;
    if (k2 == 0) {
      F[0] = F[1] = F[2] = cx(R(0), R(0));
    } else {
      const R rk2 = R(1) / R(k2);
      const R kxr = R(kx), kyr = R(ky), kzr = R(kz);
      const Cx<R> kd = scale(scale(F[0], kxr) + scale(F[1], kyr) + scale(F[2], kzr), rk2);
      F[0] = F[0] - scale(kd, kxr);
      F[1] = F[1] - scale(kd, kyr);
      F[2] = F[2] - scale(kd, kzr);
    }
    R eh = R(1), edt = R(1);
    if (op_uses_etab(OP)) { eh = a.eh[k2]; edt = a.edt[k2]; }
    const R dt = a.dt;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long o0 = c * a.lo0.cs + io0, o1 = c * a.lo1.cs + io1;
      const long long i0 = c * a.li0.cs + ii0, i1 = c * a.li1.cs + ii1;
      Cx<R> N = F[c];
      Cx<R> O = cx(R(0), R(0));
      if (op_forced(OP) && a.force != nullptr && k2 >= 4 && k2 <= 9)
        O = a.force[c * 196 + ((kx + 3) * 7 + (ky + 3)) * 4 + kz];
      if (OP != OP_HEUN1) N = N + O;  // RK4 slopes N + O (zero for the other ops)
      if (OP == OP_STORE) {
        a.out0[o0] = N;
      } else if (OP == OP_AVG) {
        a.out0[o0] = scale(a.in1[i1] + N, R(0.5));
      } else if (OP == OP_HEUN1) {
        const Cx<R> s0 = a.in0[i0];
        a.out1[o1] = scale(s0 + scale(N + O, dt), edt);
        a.out0[o0] = scale(s0, edt) + scale(N + O + O, R(0.5) * dt * eh);
      } else if (OP == OP_HEUN2) {
        a.out0[o0] = a.in1[i1] + scale(N, R(0.5) * dt * eh);
      } else if (OP == OP_EX1B) {
        const Cx<R> s0 = a.in0[i0];
        a.out0[o0] = scale(s0 + scale(a.in1[i1] + N, R(0.5) * dt * a.w), eh);
      } else if (OP == OP_EX2B) {
        const Cx<R> s0 = a.in0[i0];
        a.out0[o0] = scale(s0, edt) + scale(a.in1[i1] + N, dt * a.w * eh);
      } else if (OP == OP_RK4_0) {
        const Cx<R> s0 = a.in0[i0];
        a.out1[o1] = scale(s0 + scale(N, R(0.5) * dt), eh);
        a.out0[o0] = scale(s0 + scale(N, dt / R(6)), edt);
      } else if (OP == OP_RK4_1) {
        const Cx<R> s0 = a.in0[i0];
        a.out1[o1] = scale(s0, eh) + scale(N, R(0.5) * dt);
        a.out0[o0] = a.in1[i1] + scale(N, dt / R(3) * eh);
      } else if (OP == OP_RK4_2) {
        const Cx<R> s0 = a.in0[i0];
        a.out1[o1] = scale(s0, edt) + scale(N, dt * eh);
        a.out0[o0] = a.in1[i1] + scale(N, dt / R(3) * eh);
      } else if (OP == OP_RK4_3) {
        a.out0[o0] = a.in1[i1] + scale(N, dt / R(6));
      } else if (OP == OP_ACC) {
        a.out0[o0] = a.in1[i1] + N;
      } else if (OP == OP_MID1) {
        a.out0[o0] = scale(a.in0[i0] + scale(N, R(0.5) * dt), eh);
      } else if (OP == OP_MID2) {
        a.out0[o0] = scale(a.in0[i0], edt) + scale(N, dt * eh);
      } else if (OP == OP_EUL) {
        a.out0[o0] = scale(a.in0[i0] + scale(N, dt), edt);
      } else {  // OP_EULAV
        a.out0[o0] = scale(a.in0[i0] + scale(a.in1[i1] + N, dt * a.w), edt);
      }
    }
  }
}

// ------------------------------------------------------------------ tables
// Integrating factors exp(-nu k^2 tau) for tau = dt/2 and dt, FP64 exp, rounded once.
template <typename R>
__global__ void k_etab(R* eh, R* edt, long long k2top, double nu, double dt) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > k2top) return;
  eh[t] = R(exp(-nu * (double)t * 0.5 * dt));
  edt[t] = R(exp(-nu * (double)t * dt));
}

}  // namespace ns
