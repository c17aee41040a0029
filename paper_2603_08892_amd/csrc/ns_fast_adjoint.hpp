// ns_fast_adjoint.hpp -- specialised FP32 passes of the transposed linearised
// nonlinear term (gfx950), for the sizes of ns_fast.hpp.  Same operations and
// scratch fields as the size-generic kernels of ns_adjoint.hpp:
//   M conj(phi) [ FFT(omega x lt) + i k x FFT(lt x u) ],
//   u = IFFT(phi M a), omega = IFFT(i k x phi M a), lt = IFFT(phi P M lam);
// the velocity fields come from f_xinv and the y passes from f_ypass (9 fields
// inverse, 6 forward); this file adds the lam x pass, the z pass and the
// forward x pass with the adjoint stage combination.
#pragma once

#include "ns_adjoint.hpp"
#include "ns_fast.hpp"

namespace ns {

// ------------------------------------------------------------------ lam x pass
// lam_in = cA E_A(k) A + cB E_B(k) B on the retained modes, projected and shifted,
// inverse x transforms into scratch fields 6, 7, 8 (tiles as f_xinv).
template <typename C>
__global__ void __launch_bounds__(kFastL * C::TPL)
f_xlam(LamArgs<float> la, Cx<float>* __restrict__ W, const Cx<float>* __restrict__ twg, Shift sh,
       const int2* __restrict__ tiles, Geom g) {
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
  Cx<float> phyz = cx(1.f, 0.f);
  if (sh.on) {
    phase_row(phx, N, sh.s[0], tid, kFastL * TPL);
    phase_cols(phc, ky, kz0, sh, N, tid);
    __syncthreads();
    phyz = phc[l];
  }
  const bool col = kz < g.kzn;
  const LineTest keep = line_test(g, ky, kz);
  const LineView<float, kFastLp> lv{xb + l};
  Cx<float> q[3][EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int p = F::in_at(t, i);
    const int kx = kval(p, N);
    const bool ok = col && F::in_ok(t, i) && keep(kx);
    const int k2 = ok ? kx * kx + ky * ky + kz * kz : 0;
    const float fa = la.cA * (la.eA ? la.eA[k2] : 1.f);
    const uint32_t ia = (uint32_t)((p * N + yi) * la.la.pitch + kz);
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c][i] = scale(ld_masked(la.A + c * la.la.cs, ia, ok), fa);
    if (la.B != nullptr) {
      const float fb = la.cB * (la.eB ? la.eB[k2] : 1.f);
      const uint32_t ib = (uint32_t)((p * N + yi) * la.lb.pitch + kz);
#pragma unroll
      for (int c = 0; c < 3; ++c) q[c][i] = q[c][i] + scale(ld_masked(la.B + c * la.lb.cs, ib, ok), fb);
    }
    if (k2 == 0) {
      q[0][i] = q[1][i] = q[2][i] = cx(0.f, 0.f);
    } else {
      const float rk2 = 1.f / float(k2);
      const float kxr = float(kx), kyr = float(ky), kzr = float(kz);
      const Cx<float> kd = scale(scale(q[0][i], kxr) + scale(q[1][i], kyr) + scale(q[2][i], kzr), rk2);
      q[0][i] = q[0][i] - scale(kd, kxr);
      q[1][i] = q[1][i] - scale(kd, kyr);
      q[2][i] = q[2][i] - scale(kd, kzr);
    }
    if (sh.on) {
      const Cx<float> phi = cmul(phx[p], phyz);
#pragma unroll
      for (int c = 0; c < 3; ++c) q[c][i] = cmul(q[c][i], phi);
    }
  }
  const uint32_t obase = (uint32_t)(yi * g.kzp + kz0) + l, ostep = (uint32_t)(N * g.kzp);
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    F::run(q[f], t, lv, tw);
    if (col) {
#pragma unroll
      for (int i = 0; i < EPT; ++i)
        if (F::out_ok(t, i)) st_off(W + (6 + f) * g.wcomp, (uint32_t)F::out_pos(t, i) * ostep + obase, q[f][i]);
    }
  }
}

// ------------------------------------------------------------------ z pass
// P lines per block, TPL threads per line (block barriers when a line straddles
// wavefronts).  Inverse slices
// (u_x + i u_y), (u_z + i w_x), (w_y + i w_z), (l_x + i l_y), (l_z + i 0) from the
// half spectra of fields 0..8; the products g1 = omega x lt and g2 = lt x u stay
// in registers; forward slices (g1x + i g1y), (g1z + i g2x), (g2y + i g2z), each
// split by the line's own threads into fields 0..5 = g1x, g1y, g1z, g2x, g2y, g2z.
template <typename C, int P>
__global__ void __launch_bounds__(P * C::TPL)
f_zadj(Cx<float>* __restrict__ W, const Cx<float>* __restrict__ twg, Geom g) {
  constexpr int N = C::N, TPL = C::TPL, EPT = C::EPT, HN = N / 2, NT = P * TPL;
  using FI = RegFft<N, TPL, +1, typename C::Inv>;
  using FF = RegFft<N, TPL, -1, typename C::Fwd>;
  static_assert(FI::RL == FF::R0, "the forward transform must start with the last inverse radix");
  constexpr bool WV = (64 % TPL == 0);  // else a line straddles wavefronts: block barriers
  constexpr int LP = line_pitch(N);
  __shared__ Cx<float> tw[N];
  __shared__ Cx<float> xb[P * LP];  // exchanges
  __shared__ Cx<float> sp[P * N];   // one forward spectrum per line
  const int tid = threadIdx.x;
  const int p = tid / TPL, t = tid % TPL;
  const uint32_t line = (uint32_t)blockIdx.x * P + p;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  __syncthreads();  // the transforms below synchronise only within a wavefront
  const LineView<float, 1> lv{xb + p * LP};
  const uint32_t lbase = line * (uint32_t)g.kzp;
  Cx<float> z[4][EPT], v[EPT];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int pos = FI::in_at(t, i);
      const int k = pos <= HN ? pos : N - pos;
      const Cx<float> a = ld_masked(W + (2 * q) * g.wcomp, lbase + k, k < g.kzn);
      const Cx<float> bb = q < 4 ? ld_masked(W + (2 * q + 1) * g.wcomp, lbase + k, k < g.kzn) : cx(0.f, 0.f);
      if (pos == 0 || pos == HN) v[i] = cx(a.re, bb.re);
      else if (pos < HN) v[i] = cx(a.re - bb.im, a.im + bb.re);
      else v[i] = cx(a.re + bb.im, bb.re - a.im);
    }
    FI::template run<WV>(v, t, lv, tw);
    if (q < 4) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) z[q][i] = v[i];
    }
  }
  float g1[3][EPT], g2[3][EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const float ux = z[0][i].re, uy = z[0][i].im, uz = z[1][i].re, wx = z[1][i].im;
    const float wy = z[2][i].re, wz = z[2][i].im, lx = z[3][i].re, ly = z[3][i].im, lz = v[i].re;
    g1[0][i] = wy * lz - wz * ly;
    g1[1][i] = wz * lx - wx * lz;
    g1[2][i] = wx * ly - wy * lx;
    g2[0][i] = ly * uz - lz * uy;
    g2[1][i] = lz * ux - lx * uz;
    g2[2][i] = lx * uy - ly * ux;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const float re = q == 0 ? g1[0][i] : (q == 1 ? g1[2][i] : g2[1][i]);
      const float im = q == 0 ? g1[1][i] : (q == 1 ? g2[0][i] : g2[2][i]);
      v[i] = cx(re, im);
    }
    FF::template run<WV>(v, t, lv, tw);
    exchange_barrier<WV>();  // the previous slice's split has read sp
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (FF::out_ok(t, i)) sp[p * N + FF::out_pos(t, i)] = v[i];
    exchange_barrier<WV>();
    for (int k = t; k < g.kzn; k += TPL) {
      const Cx<float> c1 = sp[p * N + k], c2 = sp[p * N + ((N - k) % N)];
      const uint32_t off = lbase + k;
      st_off(W + (2 * q) * g.wcomp, off, cx(0.5f * (c1.re + c2.re), 0.5f * (c1.im - c2.im)));
      st_off(W + (2 * q + 1) * g.wcomp, off, cx(0.5f * (c1.im + c2.im), -0.5f * (c1.re - c2.re)));
    }
  }
}

// ------------------------------------------------------------------ forward x pass
// V = M conj(phi) (g1 + i k x g2) / N^3 from fields 0..5, then the adjoint stage
// combination AOP (tiles as f_xfwd; full mode covers every tile and writes zeros
// outside the retained set).
template <typename C, int AOP>
__global__ void __launch_bounds__(kFastL * C::TPL)
f_xadj(const Cx<float>* __restrict__ W, const Cx<float>* __restrict__ twg, Shift sh,
       const int2* __restrict__ tiles, Geom g, AdjArgs<float> a) {
  constexpr int N = C::N, TPL = C::TPL, EPT = C::EPT;
  using F = RegFft<N, TPL, -1, typename C::Fwd>;
  __shared__ Cx<float> tw[N];
  __shared__ Cx<float> phx[N];
  __shared__ Cx<float> phc[kFastL];
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
  Cx<float> r[3][EPT], v[EPT];
  Cx<float> phyz = cx(1.f, 0.f);
  if (active) {
    for (int i = tid; i < N; i += kFastL * TPL) tw[i] = twg[i];
    if (sh.on) {
      phase_row(phx, N, sh.s[0], tid, kFastL * TPL);
      phase_cols(phc, ky, kz0, sh, N, tid);
    }
    const bool col = kz < g.kzn;
    const uint32_t wbase = (uint32_t)(yi * g.kzp + kz0) + l, wstep = (uint32_t)(N * g.kzp);
    const float kyf = float(ky), kzf = float(kz);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      Cx<float>* dst = f < 3 ? r[f] : v;
#pragma unroll
      for (int i = 0; i < EPT; ++i)
        dst[i] = ld_masked(W + f * g.wcomp, (uint32_t)F::in_at(t, i) * wstep + wbase, col && F::in_ok(t, i));
      F::run(dst, t, lv, tw);  // its barriers also publish phx and phc
      if (f >= 3) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
          const float kxf = float(kval(F::out_at(t, i), N));
          const Cx<float> iv = mul_i(v[i]);
          if (f == 3) {         // i k x (g2x, 0, 0) = (0, i kz g2x, -i ky g2x)
            r[1][i] = r[1][i] + scale(iv, kzf);
            r[2][i] = r[2][i] - scale(iv, kyf);
          } else if (f == 4) {  // i k x (0, g2y, 0) = (-i kz g2y, 0, i kx g2y)
            r[0][i] = r[0][i] - scale(iv, kzf);
            r[2][i] = r[2][i] + scale(iv, kxf);
          } else {              // i k x (0, 0, g2z) = (i ky g2z, -i kx g2z, 0)
            r[0][i] = r[0][i] + scale(iv, kyf);
            r[1][i] = r[1][i] - scale(iv, kxf);
          }
        }
      }
    }
    if (sh.on) phyz = phc[l];
  }
  if (kz >= g.h || (!a.full && kz >= g.kzn)) return;
  const LineTest keep = line_test(g, ky, kz);
  const bool line_kept = active && kz < g.kzn;
  const float inv_n3 = 1.f / (float(N) * float(N) * float(N));
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    if (!F::out_ok(t, i)) continue;  // no point in this register
    const int p = F::out_pos(t, i);
    const int kx = kval(p, N);
    const uint32_t io0 = (uint32_t)((p * N + yi) * a.lo0.pitch + kz);
    if (!(line_kept && keep(kx))) {
      if (a.full)
        for (int c = 0; c < 3; ++c) st_off(a.out0 + c * a.lo0.cs, io0, cx(0.f, 0.f));
      continue;
    }
    Cx<float> V[3] = {scale(r[0][i], inv_n3), scale(r[1][i], inv_n3), scale(r[2][i], inv_n3)};
    if (sh.on) {
      const Cx<float> phi = cmul(phx[p], phyz);
#pragma unroll
      for (int c = 0; c < 3; ++c) V[c] = cmulc(V[c], phi);
    }
    const int k2 = kx * kx + ky * ky + kz * kz;
    const float eh = a.eh[k2], edt = a.edt[k2];
    const uint32_t ii0 = (uint32_t)((p * N + yi) * a.li0.pitch + kz);
    const uint32_t ii1 = (uint32_t)((p * N + yi) * a.li1.pitch + kz);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Cx<float>* out0 = a.out0 + c * a.lo0.cs;
      if (AOP == AOP_STORE) {
        st_off(out0, io0, V[c]);
      } else if (AOP == AOP_ACC) {
        st_off(out0, io0, a.in1[c * a.li1.cs + ii1] + V[c]);
      } else if (AOP == AOP_HEUN) {
        st_off(out0, io0, scale(a.in0[c * a.li0.cs + ii0] + a.in1[c * a.li1.cs + ii1], edt) + V[c]);
      } else {  // AOP_EXACT
        st_off(out0, io0, scale(a.in0[c * a.li0.cs + ii0], edt) + scale(a.in1[c * a.li1.cs + ii1], eh) + V[c]);
      }
    }
  }
}

}  // namespace ns
