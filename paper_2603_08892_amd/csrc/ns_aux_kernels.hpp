// ns_aux_kernels.hpp -- FP64 spectra reduction and the large-scale forcing draw (gfx950).
#pragma once

#include "ns_kernels.hpp"
#include "ns_aux_types.hpp"

namespace ns {

// Shell of an integer |k|^2: smallest n with n(n+1) >= k^2, i.e. n(n-1) < k^2 <= n(n+1).
__device__ __forceinline__ int shell_of(long long k2) {
  const int r = isqrt_ll(k2);
  return ((long long)r * (r + 1) >= k2) ? r : r + 1;
}

// Bin layout of one partial: [0, nsh) E, [nsh, 2nsh) D, [2nsh, 3nsh) T,
// then 3 x h one-dimensional energies, then totals E, eps, H, T, nonfinite.
// Pass 1: every wavefront takes whole k_z rows (fixed k_x, k_y) in a grid-stride
// loop, lanes along k_z, and adds into its own FP64 bins in LDS in a fixed order;
// the block then sums its wavefronts' bins in wavefront order, so the spectra are
// reproducible bit for bit.  Along a row the shell index does not decrease with
// k_z, so a segmented shuffle scan leaves each shell's sum over the 64 lanes in
// the segment's last lane, which adds it to the bin (the tails of one scan have
// distinct shells); each lane owns its k_z bin; the row total goes to its k_x and
// k_y bins from lane 0.
template <typename R>
__global__ void __launch_bounds__(1024)
k_spectra(const Cx<R>* __restrict__ u, const Cx<R>* __restrict__ nh, double nu, int n, int h,
          int nsh, long long comp, double* __restrict__ partials) {
  extern __shared__ double bins_all[];
  const int nb = 3 * nsh + 3 * h + 5;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwb = blockDim.x >> 6;
  double* bins = bins_all + wave * nb;
  for (int t = threadIdx.x; t < nwb * nb; t += blockDim.x) bins_all[t] = 0.0;
  __syncthreads();
  double tE = 0, tD = 0, tH = 0, tT = 0;
  unsigned bad = 0;
  const long long nrows = (long long)n * n;
  const long long nwaves = (long long)gridDim.x * nwb;
  for (long long row = (long long)blockIdx.x * nwb + wave; row < nrows; row += nwaves) {
    const int yi = (int)(row % n), xi = (int)(row / n);
    const int kx = kval(xi, n), ky = kval(yi, n);
    double erow = 0.0;
    for (int kz0 = 0; kz0 < h; kz0 += 64) {
      const int kz = kz0 + lane;
      const bool in = kz < h;
      double e = 0.0, d = 0.0, t = 0.0;
      int s = 0x7fffffff;  // lanes past the row end: a key above every shell
      if (in) {
        const long long idx = row * h + kz;
        const double w = (kz == 0 || 2 * kz == n) ? 1.0 : 2.0;
        const Cx<R> a0 = u[idx], a1 = u[comp + idx], a2 = u[2 * comp + idx];
        const double ar[3] = {(double)a0.re, (double)a1.re, (double)a2.re};
        const double ai[3] = {(double)a0.im, (double)a1.im, (double)a2.im};
        bool fin = true;
        for (int c = 0; c < 3; ++c) fin = fin && isfinite(ar[c]) && isfinite(ai[c]);
        if (nh != nullptr) {
          for (int c = 0; c < 3; ++c) {
            const Cx<R> b = nh[c * comp + idx];
            fin = fin && isfinite((double)b.re) && isfinite((double)b.im);
            t += ar[c] * (double)b.re + ai[c] * (double)b.im;
          }
          t *= w;
        }
        const long long k2 = (long long)kx * kx + (long long)ky * ky + (long long)kz * kz;
        s = shell_of(k2);  // kept for non-finite lanes too, so the keys stay sorted
        if (!fin) {
          ++bad;
          t = 0.0;
        } else {
          e = 0.5 * w * (ar[0] * ar[0] + ai[0] * ai[0] + ar[1] * ar[1] + ai[1] * ai[1] +
                         ar[2] * ar[2] + ai[2] * ai[2]);
          d = 2.0 * nu * (double)k2 * e;
          // helicity density: with u = a + i b, Re(conj(u).(i k x u)) = 2 k.(a x b), so
          // 1/2 w Re(conj(u).omega) = w k.(a x b)
          const double cxr = ar[1] * ai[2] - ar[2] * ai[1];
          const double cyr = ar[2] * ai[0] - ar[0] * ai[2];
          const double czr = ar[0] * ai[1] - ar[1] * ai[0];
          tH += w * ((double)kx * cxr + (double)ky * cyr + (double)kz * czr);
          tE += e;
          tD += d;
          tT += t;
          erow += e;
          bins[3 * nsh + 2 * h + kz] += e;
        }
      }
      // an iteration whose contributions are all zero changes no shell bin (skipped)
      if (__ballot(e != 0.0 || d != 0.0 || t != 0.0) == 0) continue;
      // segmented inclusive scan over the lanes (keys s non-decreasing with the lane)
      for (int off = 1; off < 64; off <<= 1) {
        const double eu = __shfl_up(e, off), du = __shfl_up(d, off);
        const int su = __shfl_up(s, off);
        double tu = 0.0;
        if (nh != nullptr) tu = __shfl_up(t, off);
        if (lane >= off && su == s) {
          e += eu;
          d += du;
          t += tu;
        }
      }
      const int sn = __shfl_down(s, 1);
      if (in && (lane == 63 || sn != s)) {
        bins[s] += e;
        bins[nsh + s] += d;
        if (nh != nullptr) bins[2 * nsh + s] += t;
      }
    }
    for (int off = 32; off > 0; off >>= 1) erow += __shfl_down(erow, off);
    if (lane == 0) {
      bins[3 * nsh + abs(kx)] += erow;
      bins[3 * nsh + h + abs(ky)] += erow;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    tE += __shfl_down(tE, off);
    tD += __shfl_down(tD, off);
    tH += __shfl_down(tH, off);
    tT += __shfl_down(tT, off);
    bad += __shfl_down(bad, off);
  }
  const int tot = 3 * nsh + 3 * h;
  if (lane == 0) {
    bins[tot + 0] = tE;
    bins[tot + 1] = tD;
    bins[tot + 2] = tH;
    bins[tot + 3] = tT;
    bins[tot + 4] = (double)bad;
  }
  __syncthreads();
  double* out = partials + (long long)blockIdx.x * nb;
  for (int t = threadIdx.x; t < nb; t += blockDim.x) {
    double acc = 0.0;
    for (int w = 0; w < nwb; ++w) acc += bins_all[w * nb + t];
    out[t] = acc;
  }
}

// Pass 2: fixed-order sum over the blocks' partials.  Eight bins per block of 256
// threads; the 32 lanes of a bin sum the partials b = lane, lane + 32, ... in
// order, then a fixed shuffle tree combines the lanes (deterministic).
__global__ void __launch_bounds__(256)
k_spectra_sum(const double* __restrict__ partials, int nblocks, int nb, double* __restrict__ out) {
  const int bin = blockIdx.x * 8 + (threadIdx.x >> 5);
  const int lane = threadIdx.x & 31;
  double s = 0.0;
  if (bin < nb)
    for (int b = lane; b < nblocks; b += 32) s += partials[(long long)b * nb + bin];
  for (int off = 16; off > 0; off >>= 1) s += __shfl_down(s, off, 32);
  if (lane == 0 && bin < nb) out[bin] = s;
}

// ------------------------------------------------------------------ forcing
// SplitMix64 (Steele, Lea & Flood 2014) used counter-based:
// stream(seed, step) = mix(seed + G (step + 1)), draw j = mix(stream + G (j + 1)),
// uniform = (draw >> 11) 2^-53; Box-Muller on pairs (u1, u2).
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double sm64_uniform(uint64_t seed, long long step, long long j) {
  const uint64_t G = 0x9E3779B97F4A7C15ull;
  const uint64_t s = sm64_mix(seed + G * (uint64_t)(step + 1));
  return (double)(sm64_mix(s + G * (uint64_t)(j + 1)) >> 11) * (1.0 / 9007199254740992.0);
}

// Forced modes 4 <= |k|^2 <= 9 in draw order (k_z 0..3, then k_x, k_y from -3 to 3;
// on k_z = 0 only k_x > 0, or k_x = 0 and k_y > 0): 48 independent modes, listed at
// compile time.
struct ForcingModes {
  int k[48][3];
};
constexpr ForcingModes make_forcing_modes() {
  ForcingModes m{};
  int c = 0;
  for (int z = 0; z <= 3; ++z)
    for (int x = -3; x <= 3; ++x)
      for (int y = -3; y <= 3; ++y) {
        const int k2 = x * x + y * y + z * z;
        if (k2 < 4 || k2 > 9) continue;
        if (z == 0 && !(x > 0 || (x == 0 && y > 0))) continue;
        m.k[c][0] = x;
        m.k[c][1] = y;
        m.k[c][2] = z;
        ++c;
      }
  return m;
}
__device__ __forceinline__ void forcing_mode(int i, int* kx, int* ky, int* kz) {
  constexpr ForcingModes m = make_forcing_modes();
  static_assert(m.k[47][2] == 3 && m.k[0][2] == 0, "48 forced modes");
  *kx = m.k[i][0];
  *ky = m.k[i][1];
  *kz = m.k[i][2];
}

// One block of 192 threads: draw g for `step` (thread 3 i + c the Gaussian pair of
// mode i, component c), project it, scale it to inject energy at rate `inj` over a
// step dt from state u, write the dense table force[c][k_x+3][k_y+3][k_z] (k_z <= 3)
// and the FP64 record fs.
template <typename R>
__global__ void __launch_bounds__(192)
k_forcing(const Cx<R>* __restrict__ u, Cx<R>* __restrict__ force, ForceState* __restrict__ fs, int n,
          int pitch, long long comp, uint64_t seed, long long step, double dt, double inj) {
  __shared__ double gre[48][3], gim[48][3], pb[48], pg[48];
  __shared__ double amp;
  const int q = threadIdx.x;
  for (int t = q; t < 3 * 196; t += blockDim.x) force[t] = cx(R(0), R(0));
  if (q < 144) {
    const long long p = q;  // = 3 i + c
    const double u1 = sm64_uniform(seed, step, 2 * p);
    const double u2 = sm64_uniform(seed, step, 2 * p + 1);
    const double r = sqrt(-2.0 * log(1.0 - u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    gre[q / 3][q % 3] = r * cs;
    gim[q / 3][q % 3] = r * sn;
  }
  __syncthreads();
  if (q < 48) {
    const int i = q;
    int kx, ky, kz;
    forcing_mode(i, &kx, &ky, &kz);
    double vr[3], vi[3];
    for (int c = 0; c < 3; ++c) {
      vr[c] = gre[i][c];
      vi[c] = gim[i][c];
    }
    const double k2 = (double)(kx * kx + ky * ky + kz * kz);
    const double dr = (kx * vr[0] + ky * vr[1] + kz * vr[2]) / k2;
    const double di = (kx * vi[0] + ky * vi[1] + kz * vi[2]) / k2;
    vr[0] -= kx * dr; vr[1] -= ky * dr; vr[2] -= kz * dr;
    vi[0] -= kx * di; vi[1] -= ky * di; vi[2] -= kz * di;
    // B and G contributions of the stored half-spectrum entries of this mode
    const long long idx = ((long long)((kx + n) % n) * n + (ky + n) % n) * pitch + kz;
    double b = 0, g2 = 0;
    const double w = (kz == 0) ? 1.0 : 2.0;
    for (int c = 0; c < 3; ++c) {
      const Cx<R> a = u[c * comp + idx];
      b += w * ((double)a.re * vr[c] + (double)a.im * vi[c]);
      g2 += w * (vr[c] * vr[c] + vi[c] * vi[c]);
    }
    if (kz == 0) {  // the partner -k holds conj(g)
      const long long idp = ((long long)((-kx + n) % n) * n + (-ky + n) % n) * pitch;
      for (int c = 0; c < 3; ++c) {
        const Cx<R> a = u[c * comp + idp];
        b += (double)a.re * vr[c] - (double)a.im * vi[c];
        g2 += vr[c] * vr[c] + vi[c] * vi[c];
      }
    }
    for (int c = 0; c < 3; ++c) {
      gre[i][c] = vr[c];
      gim[i][c] = vi[c];
      fs->g[i][c][0] = vr[c];
      fs->g[i][c][1] = vi[c];
    }
    pb[i] = b;
    pg[i] = g2;
  }
  __syncthreads();
  if (q == 0) {
    double B = 0, G = 0;
    for (int m = 0; m < 48; ++m) { B += pb[m]; G += pg[m]; }
    const double r = sqrt(B * B + 2.0 * dt * G * inj);
    amp = 2.0 * inj / (B + r);
    fs->amp = amp;
    fs->B = B;
    fs->G = G;
    fs->r = r;
    fs->injected = dt * (amp * B + 0.5 * amp * amp * dt * G);
  }
  __syncthreads();
  if (q < 144) {
    const int i = q / 3, c = q % 3;
    int kx, ky, kz;
    forcing_mode(i, &kx, &ky, &kz);
    const double re = amp * gre[i][c], im = amp * gim[i][c];
    force[c * 196 + ((kx + 3) * 7 + (ky + 3)) * 4 + kz] = cx(R(re), R(im));
    if (kz == 0) force[c * 196 + ((-kx + 3) * 7 + (-ky + 3)) * 4] = cx(R(re), R(-im));
  }
}

// ------------------------------------------------------------------ forced step adjoint
// The forcing O = a(u0) g depends on the state through B = <u0, g> (the
// amplitude solves a B + a^2 dt/2 G = inj), with da/dB = -a/r.  With
// mu_O = (dS_new/dO)^T lam = dt (E_h lam + E_dt mu1) for the Heun step (mu1 the
// adjoint of the first stage), the step adjoint gains (da/dB) <mu_O, g> g.
// k_forcing_adj_dot (one block, before lam is overwritten) forms the scalar
// (da/dB) <mu_O, g> over the 96 forced full-grid modes (Parseval weights: 2 off
// the k_z = 0 plane, 1 on it, where both k and -k are stored); k_forcing_adj_add
// adds it times g to the result.
template <typename R>
__global__ void __launch_bounds__(64)
k_forcing_adj_dot(const Cx<R>* __restrict__ lam, Lay ll, const Cx<R>* __restrict__ mu1, Lay lm,
                  const R* __restrict__ eh, const R* __restrict__ edt, ForceState* __restrict__ fs, int n,
                  double dt) {
  __shared__ double part[64];
  const int i = threadIdx.x;
  double acc = 0.0;
  if (i < 48) {
    int kx, ky, kz;
    forcing_mode(i, &kx, &ky, &kz);
    const int k2 = kx * kx + ky * ky + kz * kz;
    const double fh = (double)eh[k2], fd = (double)edt[k2];
    for (int side = 0; side < (kz == 0 ? 2 : 1); ++side) {
      const int sx = side ? -kx : kx, sy = side ? -ky : ky;
      const int xi = (sx + n) % n, yi = (sy + n) % n;
      const double w = (kz == 0) ? 1.0 : 2.0;
      for (int c = 0; c < 3; ++c) {
        const Cx<R> l = lam[c * ll.cs + lay_at(ll, xi, yi, kz, n)];
        const Cx<R> m = mu1[c * lm.cs + lay_at(lm, xi, yi, kz, n)];
        const double mre = dt * (fh * (double)l.re + fd * (double)m.re);
        const double mim = dt * (fh * (double)l.im + fd * (double)m.im);
        const double gre = fs->g[i][c][0], gim = side ? -fs->g[i][c][1] : fs->g[i][c][1];
        acc += w * (mre * gre + mim * gim);
      }
    }
  }
  part[i] = acc;
  __syncthreads();
  if (i == 0) {
    double t = 0.0;
    for (int m = 0; m < 48; ++m) t += part[m];
    fs->dot = -(fs->amp / fs->r) * t;
  }
}

template <typename R>
__global__ void __launch_bounds__(64)
k_forcing_adj_add(Cx<R>* __restrict__ lam, Lay ll, const ForceState* __restrict__ fs, int n) {
  const int i = threadIdx.x;
  if (i >= 48) return;
  int kx, ky, kz;
  forcing_mode(i, &kx, &ky, &kz);
  const double s = fs->dot;
  for (int side = 0; side < (kz == 0 ? 2 : 1); ++side) {
    const int sx = side ? -kx : kx, sy = side ? -ky : ky;
    const int xi = (sx + n) % n, yi = (sy + n) % n;
    for (int c = 0; c < 3; ++c) {
      const long long o = c * ll.cs + lay_at(ll, xi, yi, kz, n);
      const double gre = fs->g[i][c][0], gim = side ? -fs->g[i][c][1] : fs->g[i][c][1];
      const Cx<R> v = lam[o];
      lam[o] = cx(R((double)v.re + s * gre), R((double)v.im + s * gim));
    }
  }
}

// ------------------------------------------------------------------ energy budget
// Pass 1: E = 1/2 sum w |u|^2 and eps = nu sum w |k|^2 |u|^2 over the retained
// modes of a state (any layout; entries outside the retained set are ignored),
// per block in a fixed order: every wavefront takes whole (k_x, k_y) rows in a
// grid-stride loop (rows whose k_z = 0 mode is not retained hold no retained mode
// and are skipped), lanes along k_z < kzn; a shuffle tree per wavefront, then the
// wavefronts in order.
constexpr int kBudgetBlocks = 1024;
template <typename R>
__global__ void __launch_bounds__(256)
k_budget_partial(const Cx<R>* __restrict__ u, Lay lu, Geom g, double nu, double* __restrict__ partials) {
  __shared__ double we[4], wd[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nrows = g.n * g.n, nwaves = gridDim.x * 4;
  double e = 0.0, d = 0.0;
  for (int row = blockIdx.x * 4 + wave; row < nrows; row += nwaves) {
    const int xi = row / g.n, yi = row - xi * g.n;
    const int kx = kval(xi, g.n), ky = kval(yi, g.n);
    if (!retained(g, kx, ky, 0)) continue;  // the same for the whole wavefront
    const long long base = lay_at(lu, xi, yi, 0, g.n);
    for (int kz = lane; kz < g.kzn; kz += 64) {
      if (!retained(g, kx, ky, kz)) continue;
      const double w = (kz == 0 || 2 * kz == g.n) ? 1.0 : 2.0;
      double m2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        const Cx<R> a = u[c * lu.cs + base + kz];
        m2 += (double)a.re * (double)a.re + (double)a.im * (double)a.im;
      }
      const double em = 0.5 * w * m2;
      e += em;
      d += 2.0 * nu * (double)((long long)kx * kx + (long long)ky * ky + (long long)kz * kz) * em;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_down(e, off);
    d += __shfl_down(d, off);
  }
  if (lane == 0) {
    we[wave] = e;
    wd[wave] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = ((we[0] + we[1]) + we[2]) + we[3];
    partials[2 * blockIdx.x + 1] = ((wd[0] + wd[1]) + wd[2]) + wd[3];
  }
}

// Pass 2 (one wavefront): sum the partials in a fixed order and update the
// record.  dt == 0 starts the budget at this state.  forced: add the injected
// energy of the step from the forcing record.
__global__ void __launch_bounds__(64)
k_budget_step(const double* __restrict__ partials, int nblocks, Budget* __restrict__ b,
              const ForceState* __restrict__ fs, double dt, int forced) {
  const int lane = threadIdx.x;
  double e = 0.0, d = 0.0;
  for (int k = lane; k < nblocks; k += 64) {
    e += partials[2 * k];
    d += partials[2 * k + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_down(e, off);
    d += __shfl_down(d, off);
  }
  if (lane != 0) return;
  if (dt == 0.0) {
    b->t = 0.0;
    b->E0 = e;
    b->int_eps = 0.0;
    b->int_p = 0.0;
    b->p_last = 0.0;
  } else {
    b->t += dt;
    b->int_eps += 0.5 * dt * (b->eps + d);
    const double inj = forced ? fs->injected : 0.0;
    b->int_p += inj;
    b->p_last = inj / dt;
  }
  b->E = e;
  b->eps = d;
  b->residual = e - b->E0 + b->int_eps - b->int_p;
}

}  // namespace ns
