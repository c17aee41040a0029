// The one-dimensional quadratic model dS/dt = -S^2 used to illustrate the time
// schemes (Sec. "Phase shifting for one-dimensional problems", Eqs. model-1d-2 and
// 1d_initial, Fig. 8), FP64, for a batch of independent real signals.
//
// One block per signal; the whole signal (n <= 1024 points) and every stage of a
// step live in LDS, so a launch advances the signal by all its steps with no HBM
// traffic between stages.  The transforms are direct sums with exact integer
// twiddle indices ((k j) mod n): the signals are short and the cost O(n k_max)
// per transform is immaterial next to the launch.
//
//   N(S; s)_k = M_k conj(phi_k) (1/n) sum_j w_j e^{-2 pi i k j / n},
//   w_j = -v_j^2,  v_j = sum_k (phi M S)_k e^{2 pi i k j / n} (real field, Hermitian),
//   phi_k = e^{2 pi i k s / n},  M_k = [k <= kmax].
#pragma once

#include <hip/hip_runtime.h>

namespace ns1d {

enum Scheme { EULER = 0, EULER_PS = 1, RK2 = 2, PS_EXACT = 3, PS_APPROX = 4, RK4 = 5 };

struct Args {
  const double2* in;   // [batch][h] input spectra
  double2* out;        // [batch][h] result (may alias in)
  int n, h, kmax;
  double dt;
  int nsteps;
  int scheme;          // Scheme, or -1: one evaluation N(S; shift) into out
  double shift;        // grid shift in cells for scheme -1
};

constexpr int kThreads = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

struct Lds {
  double2* tw;   // [n]  e^{2 pi i m / n}
  double* v;     // [n]  grid values, then -v^2
  double2* ph;   // [h]  phase factors of the current shift
};

// out[0..h) = N(x; shift); every thread of the block takes part (barriers inside).
__device__ void evaluate(const Lds& L, const double2* x, double2* out, double shift, int n, int h, int kmax) {
  const int tid = threadIdx.x;
  for (int k = tid; k < h; k += kThreads) {
    double sn, cs;
    sincospi(2.0 * (double)k * shift / (double)n, &sn, &cs);
    L.ph[k] = make_double2(cs, sn);
  }
  __syncthreads();
  for (int j = tid; j < n; j += kThreads) {
    double acc = 0.0;
    int m = j;  // (k j) mod n for k = 1
    for (int k = 1; k <= kmax; ++k) {
      const double2 a = cmul(x[k], L.ph[k]);
      const double2 e = L.tw[m];
      acc += a.x * e.x - a.y * e.y;
      m += j;
      if (m >= n) m -= n;
    }
    const double v = x[0].x + 2.0 * acc;  // the k = 0 coefficient of a real field is real
    L.v[j] = -v * v;
  }
  __syncthreads();
  const double inv_n = 1.0 / (double)n;
  for (int k = tid; k < h; k += kThreads) {
    double2 r = make_double2(0.0, 0.0);
    if (k <= kmax) {
      int m = 0;
      double re = 0.0, im = 0.0;
      for (int j = 0; j < n; ++j) {
        const double2 e = L.tw[m];
        re += L.v[j] * e.x;
        im -= L.v[j] * e.y;
        m += k;
        if (m >= n) m -= n;
      }
      const double2 p = L.ph[k];
      r = make_double2((re * p.x + im * p.y) * inv_n, (im * p.x - re * p.y) * inv_n);  // conj(phi) F
    }
    out[k] = r;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kThreads) k_model1d(Args a) {
  extern __shared__ unsigned char smem_raw[];
  const int n = a.n, h = a.h, tid = threadIdx.x;
  double2* base = reinterpret_cast<double2*>(smem_raw);
  Lds L{base, reinterpret_cast<double*>(base + n), base + n + (n + 1) / 2};
  double2* s0 = L.ph + h;  // state at the start of the step
  double2* sa = s0 + h;    // stage state
  double2* n0 = sa + h;    // evaluations
  double2* n1 = n0 + h;
  double2* n2 = n1 + h;
  double2* n3 = n2 + h;
  const double2* in = a.in + (size_t)blockIdx.x * h;
  double2* out = a.out + (size_t)blockIdx.x * h;
  for (int m = tid; m < n; m += kThreads) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)n, &sn, &cs);
    L.tw[m] = make_double2(cs, sn);
  }
  for (int k = tid; k < h; k += kThreads) s0[k] = in[k];
  __syncthreads();
  if (a.scheme < 0) {
    evaluate(L, s0, n0, a.shift, n, h, a.kmax);
    for (int k = tid; k < h; k += kThreads) out[k] = n0[k];
    return;
  }
  const double dt = a.dt, hd = 0.5 * dt;
  // s = x + c y (+ d z), elementwise over the h coefficients
  auto axpy = [&](double2* s, const double2* x, double c, const double2* y) {
    for (int k = tid; k < h; k += kThreads) s[k] = make_double2(x[k].x + c * y[k].x, x[k].y + c * y[k].y);
    __syncthreads();
  };
  // two-shift average of Eq. sum_ps_non_ps into r (uses n3 as scratch)
  auto average = [&](const double2* x, double2* r) {
    evaluate(L, x, r, 0.0, n, h, a.kmax);
    evaluate(L, x, n3, 0.5, n, h, a.kmax);
    for (int k = tid; k < h; k += kThreads) r[k] = make_double2(0.5 * (r[k].x + n3[k].x), 0.5 * (r[k].y + n3[k].y));
    __syncthreads();
  };
  for (int step = 0; step < a.nsteps; ++step) {
    switch (a.scheme) {
      case EULER:
        evaluate(L, s0, n0, 0.0, n, h, a.kmax);
        axpy(s0, s0, dt, n0);
        break;
      case EULER_PS:
        average(s0, n0);
        axpy(s0, s0, dt, n0);
        break;
      case RK2:
      case PS_EXACT:
        // midpoint: S_h = S0 + dt/2 A(S0), S = S0 + dt A(S_h)
        if (a.scheme == RK2) evaluate(L, s0, n0, 0.0, n, h, a.kmax);
        else average(s0, n0);
        axpy(sa, s0, hd, n0);
        if (a.scheme == RK2) evaluate(L, sa, n1, 0.0, n, h, a.kmax);
        else average(sa, n1);
        axpy(s0, s0, dt, n1);
        break;
      case PS_APPROX:
        // Heun with shifts 0 and 1/2: S1 = S0 + dt N(S0; 0), S = S0 + dt/2 (N(S0; 0) + N(S1; 1/2))
        evaluate(L, s0, n0, 0.0, n, h, a.kmax);
        axpy(sa, s0, dt, n0);
        evaluate(L, sa, n1, 0.5, n, h, a.kmax);
        for (int k = tid; k < h; k += kThreads)
          s0[k] = make_double2(s0[k].x + hd * (n0[k].x + n1[k].x), s0[k].y + hd * (n0[k].y + n1[k].y));
        __syncthreads();
        break;
      default:  // RK4, classical (no linear term, so the Lawson form is the plain one)
        evaluate(L, s0, n0, 0.0, n, h, a.kmax);
        axpy(sa, s0, hd, n0);
        evaluate(L, sa, n1, 0.0, n, h, a.kmax);
        axpy(sa, s0, hd, n1);
        evaluate(L, sa, n2, 0.0, n, h, a.kmax);
        axpy(sa, s0, dt, n2);
        evaluate(L, sa, n3, 0.0, n, h, a.kmax);
        for (int k = tid; k < h; k += kThreads) {
          const double c = dt / 6.0;
          s0[k] = make_double2(s0[k].x + c * (n0[k].x + 2.0 * n1[k].x + 2.0 * n2[k].x + n3[k].x),
                               s0[k].y + c * (n0[k].y + 2.0 * n1[k].y + 2.0 * n2[k].y + n3[k].y));
        }
        __syncthreads();
        break;
    }
  }
  for (int k = tid; k < h; k += kThreads) out[k] = s0[k];
}

// Bytes of LDS for signal length n: tw[n], v[n] (as n/2 rounded up double2), ph and
// six h-arrays.
inline size_t lds_bytes(int n) {
  const int h = n / 2 + 1;
  return sizeof(double2) * ((size_t)n + (size_t)(n + 1) / 2 + 7 * (size_t)h);
}

}  // namespace ns1d
