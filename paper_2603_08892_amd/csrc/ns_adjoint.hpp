// ns_adjoint.hpp -- kernels of the transposed linearised nonlinear term (gfx950).
//
// With the Parseval inner product <a, b> = sum_k w Re(conj(a).b), the inverse
// transform is an isometry onto real fields, P, M and the curl are self-adjoint
// and conj(phi) is the adjoint of phi.  From a.(b x c) = b.(c x a), the transpose
// of the linearisation of N(a) = M conj(phi) P FFT(IFFT(phi M a) x IFFT(i k x phi M a))
// applied to lam is
//   M conj(phi) [ FFT(omega x lt) + i k x FFT(lt x u) ],
//   u = IFFT(phi M a), omega = IFFT(i k x phi M a), lt = IFFT(phi P M lam).
// Passes: k_xinv (velocity, 6 fields) and k_xlam (lam, 3 fields), y-inverse of 9
// fields, k_zadj (c2r of 9, the two products, r2c of 6), y-forward of 6, k_xadj.
#pragma once

#include "ns_kernels.hpp"

namespace ns {

// Input of the lam pass: lam_in = cA E_A(k) A + cB E_B(k) B (B, E_A, E_B optional),
// then projection, truncation and phase.
template <typename R>
struct LamArgs {
  const Cx<R>* A;
  const Cx<R>* B;
  const R* eA;
  const R* eB;
  R cA, cB;
  Lay la, lb;  // layouts of A and B
};

// ------------------------------------------------------------------ k_xlam
// Same tiling as k_xinv; writes scratch fields 6, 7, 8.
template <typename R, int EPT>
__global__ void __launch_bounds__(512)
k_xlam(LamArgs<R> la, Cx<R>* __restrict__ W, const Cx<R>* __restrict__ twg, Shift sh,
       const int2* __restrict__ tiles, Geom g, FftPlan plan) {
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
  Cx<R> v[3][EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nt;
    v[0][i] = v[1][i] = v[2][i] = cx(R(0), R(0));
    if (e < npts) {
      const int p = e >> g.lgL, l = e & (L - 1);
      const int kz = kz0 + l, kx = kval(p, n);
      if (kz < g.kzn && retained(g, kx, ky, kz)) {
        const long long ia = lay_at(la.la, p, yi, kz, n);
        const long long k2 = (long long)kx * kx + (long long)ky * ky + (long long)kz * kz;
        R fa = la.cA * (la.eA ? la.eA[k2] : R(1));
        Cx<R> q[3];
        for (int c = 0; c < 3; ++c) q[c] = scale(la.A[c * la.la.cs + ia], fa);
        if (la.B != nullptr) {
          const long long ib = lay_at(la.lb, p, yi, kz, n);
          const R fb = la.cB * (la.eB ? la.eB[k2] : R(1));
          for (int c = 0; c < 3; ++c) q[c] = q[c] + scale(la.B[c * la.lb.cs + ib], fb);
        }
        if (k2 == 0) {
          q[0] = q[1] = q[2] = cx(R(0), R(0));
        } else {
          const R rk2 = R(1) / R(k2);
          const R kxr = R(kx), kyr = R(ky), kzr = R(kz);
          const Cx<R> kd = scale(scale(q[0], kxr) + scale(q[1], kyr) + scale(q[2], kzr), rk2);
          q[0] = q[0] - scale(kd, kxr);
          q[1] = q[1] - scale(kd, kyr);
          q[2] = q[2] - scale(kd, kzr);
        }
        if (sh.on) {
          const Cx<R> phi = cmul(phx[p], cmul(phy, phase1<R>(kz, sh.s[2], n)));
          for (int c = 0; c < 3; ++c) q[c] = cmul(q[c], phi);
        }
        v[0][i] = q[0];
        v[1][i] = q[1];
        v[2][i] = q[2];
      }
    }
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nt;
      if (e < npts) buf[e] = v[f][i];
    }
    __syncthreads();
    fft_lines<+1, EPT, true>(buf, tw, plan, L, L, 1, tid, nt);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nt;
      if (e < npts) {
        const int p = e >> g.lgL, l = e & (L - 1);
        const int kz = kz0 + l;
        if (kz < g.kzn) W[(6 + f) * g.wcomp + ((long long)p * n + yi) * g.kzp + kz] = buf[e];
      }
    }
  }
}

// ------------------------------------------------------------------ k_zadj
// P (even) lines per block.  Inverse slots: 4p+0 (u_x, u_y), 4p+1 (u_z, w_x),
// 4p+2 (w_y, w_z), 4p+3 (l_x, l_y), and 4P+j (l_z of lines 2j, 2j+1).  Products
// g1 = omega x lt, g2 = lt x u; forward slots 3p+0 (g1x, g1y), 3p+1 (g1z, g2x),
// 3p+2 (g2y, g2z).  Output scratch fields 0..5 = g1x, g1y, g1z, g2x, g2y, g2z.
template <typename R, int EPT>
__global__ void __launch_bounds__(512)
k_zadj(Cx<R>* __restrict__ W, const Cx<R>* __restrict__ twg, int P, Geom g, FftPlan plan) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem_raw);
  Cx<R>* buf = tw + g.n;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = g.n, hn = n / 2;
  const long long line0 = (long long)blockIdx.x * P;
  for (int t = tid; t < n; t += nt) tw[t] = twg[t];
  const int nk = hn + 1;
  const int nslot_in = 4 * P + P / 2;
  for (int idx = tid; idx < nslot_in * nk; idx += nt) {
    const int k = idx % nk;
    const int s = idx / nk;
    Cx<R> a = cx(R(0), R(0)), bb = cx(R(0), R(0));
    if (k < g.kzn) {
      if (s < 4 * P) {
        const int p = s / 4, q = s % 4;
        const long long off = (line0 + p) * g.kzp + k;
        a = W[(2 * q) * g.wcomp + off];
        bb = W[(2 * q + 1) * g.wcomp + off];
      } else {
        const int j = s - 4 * P;
        a = W[8 * g.wcomp + (line0 + 2 * j) * g.kzp + k];
        bb = W[8 * g.wcomp + (line0 + 2 * j + 1) * g.kzp + k];
      }
    }
    Cx<R>* z = buf + s * n;
    if (k == 0 || k == hn) {
      z[k] = cx(a.re, bb.re);
    } else {
      z[k] = cx(a.re - bb.im, a.im + bb.re);
      z[n - k] = cx(a.re + bb.im, bb.re - a.im);
    }
  }
  __syncthreads();
  fft_lines<+1, EPT, false>(buf, tw, plan, nslot_in, 1, n, tid, nt);
  constexpr int PPT = (2 * EPT + 8) / 9;  // points per thread: 4.5 P n <= EPT nt
  R g1[3][PPT], g2[3][PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int e = tid + i * nt;
    if (e < P * n) {
      const int p = e / n, j = e % n;
      const Cx<R> z0 = buf[(4 * p) * n + j], z1 = buf[(4 * p + 1) * n + j];
      const Cx<R> z2 = buf[(4 * p + 2) * n + j], z3 = buf[(4 * p + 3) * n + j];
      const Cx<R> zs = buf[(4 * P + p / 2) * n + j];
      const R ux = z0.re, uy = z0.im, uz = z1.re, wx = z1.im, wy = z2.re, wz = z2.im;
      const R lx = z3.re, ly = z3.im, lz = (p & 1) ? zs.im : zs.re;
      g1[0][i] = wy * lz - wz * ly;
      g1[1][i] = wz * lx - wx * lz;
      g1[2][i] = wx * ly - wy * lx;
      g2[0][i] = ly * uz - lz * uy;
      g2[1][i] = lz * ux - lx * uz;
      g2[2][i] = lx * uy - ly * ux;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int e = tid + i * nt;
    if (e < P * n) {
      const int p = e / n, j = e % n;
      buf[(3 * p) * n + j] = cx(g1[0][i], g1[1][i]);
      buf[(3 * p + 1) * n + j] = cx(g1[2][i], g2[0][i]);
      buf[(3 * p + 2) * n + j] = cx(g2[1][i], g2[2][i]);
    }
  }
  __syncthreads();
  fft_lines<-1, EPT, false>(buf, tw, plan, 3 * P, 1, n, tid, nt);
  for (int idx = tid; idx < 3 * P * g.kzn; idx += nt) {
    const int k = idx % g.kzn, s = idx / g.kzn;
    const Cx<R> c1 = buf[s * n + k];
    const Cx<R> c2 = buf[s * n + ((n - k) % n)];
    const Cx<R> a = cx(R(0.5) * (c1.re + c2.re), R(0.5) * (c1.im - c2.im));
    const Cx<R> bb = cx(R(0.5) * (c1.im + c2.im), R(-0.5) * (c1.re - c2.re));
    const int p = s / 3, q = s % 3;
    const long long off = (line0 + p) * g.kzp + k;
    W[(2 * q) * g.wcomp + off] = a;
    W[(2 * q + 1) * g.wcomp + off] = bb;
  }
}

// ------------------------------------------------------------------ k_xadj
enum AdjOp {
  AOP_STORE = 0,  // out0 = V
  AOP_ACC = 1,    // out0 = in1 + V
  AOP_HEUN = 2,   // out0 = E_dt (in0 + in1) + V
  AOP_EXACT = 3   // out0 = E_dt in0 + E_h in1 + V
};

template <typename R>
struct AdjArgs {
  Cx<R>* out0;
  const Cx<R>* in0;
  const Cx<R>* in1;
  const R* eh;
  const R* edt;
  int full;
  int ntzf;
  Lay lo0, li0, li1;  // layouts of out0, in0, in1
};

// Forward x pass of g1 = FFT(omega x lt) and g2 = FFT(lt x u):
// V = M conj(phi) (g1 + i k x g2) / N^3, then the adjoint stage combination.
template <typename R, int EPT, int OP>
__global__ void __launch_bounds__(512)
k_xadj(const Cx<R>* __restrict__ W, const Cx<R>* __restrict__ twg, Shift sh,
       const int2* __restrict__ tiles, Geom g, FftPlan plan, AdjArgs<R> a) {
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
    for (int f = 0; f < 6; ++f) {
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
        const Cx<R> v = (e < npts) ? buf[e] : cx(R(0), R(0));
        const int p = e >> g.lgL, l = e & (L - 1);
        const R kx = R(kval(p, n)), kyr = R(ky), kz = R(kz0 + l);
        if (f < 3) {
          r[f][i] = v;
        } else if (f == 3) {  // i k x (g2x, 0, 0) = (0, i kz g2x, -i ky g2x)
          r[1][i] = r[1][i] + scale(mul_i(v), kz);
          r[2][i] = r[2][i] - scale(mul_i(v), kyr);
        } else if (f == 4) {  // i k x (0, g2y, 0) = (-i kz g2y, 0, i kx g2y)
          r[0][i] = r[0][i] - scale(mul_i(v), kz);
          r[2][i] = r[2][i] + scale(mul_i(v), kx);
        } else {  // i k x (0, 0, g2z) = (i ky g2z, -i kx g2z, 0)
          r[0][i] = r[0][i] + scale(mul_i(v), kyr);
          r[1][i] = r[1][i] - scale(mul_i(v), kx);
        }
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
      if (a.full)
        for (int c = 0; c < 3; ++c) a.out0[c * a.lo0.cs + io0] = cx(R(0), R(0));
      continue;
    }
    const long long ii0 = lay_at(a.li0, p, yi, kz, n), ii1 = lay_at(a.li1, p, yi, kz, n);
    Cx<R> V[3] = {scale(r[0][i], inv_n3), scale(r[1][i], inv_n3), scale(r[2][i], inv_n3)};
    if (sh.on) {
      const Cx<R> phi = cmul(cmul(phx[p], phase1<R>(ky, sh.s[1], n)), phase1<R>(kz, sh.s[2], n));
      for (int c = 0; c < 3; ++c) V[c] = cmulc(V[c], phi);
    }
    const long long k2 = (long long)kx * kx + (long long)ky * ky + (long long)kz * kz;
    const R eh = a.eh[k2], edt = a.edt[k2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long o = c * a.lo0.cs + io0, i0 = c * a.li0.cs + ii0, i1 = c * a.li1.cs + ii1;
      if (OP == AOP_STORE) a.out0[o] = V[c];
      else if (OP == AOP_ACC) a.out0[o] = a.in1[i1] + V[c];
      else if (OP == AOP_HEUN) a.out0[o] = scale(a.in0[i0] + a.in1[i1], edt) + V[c];
      else a.out0[o] = scale(a.in0[i0], edt) + scale(a.in1[i1], eh) + V[c];
    }
  }
}

}  // namespace ns
