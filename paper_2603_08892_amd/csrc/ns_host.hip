// ns_host.hip -- implementation of the C ABI declared in include/ns.h.
//
// Host side: argument checks, geometry of the pruned transforms, FFT plans,
// workspace layout, and the launch sequences of one nonlinear-term evaluation
// and of the Runge-Kutta schemes (Eq. base-eq integrated with exact integrating
// factors; RK4 in Lawson form, RK2 phase-shift exact / approx / random).
#include <hip/hip_runtime.h>

#include <mutex>

#include "ns_host_impl.hpp"
#include "ns_aux_kernels.hpp"
#include "ns_model1d.hpp"

namespace nsh {
thread_local std::string g_last_error;
}  // namespace nsh

using namespace nsh;

namespace {

using namespace nsh;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Largest integer strictly below x, a value within relative 1e-9 of an integer
// being taken as that integer.
long long largest_int_below(double x) {
  const double eps = 1e-9 * std::fmax(1.0, std::fabs(x));
  return (long long)std::ceil(x - eps) - 1;
}

bool factor_ok(int n, std::vector<int>* radices) {
  if (n < 8 || n > 1024) return false;
  int m = n, a = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  if (a < 1) return false;
  std::vector<int> r;
  while (a >= 3 && a != 4) { r.push_back(8); a -= 3; }
  if (a == 4) { r.push_back(4); r.push_back(4); a = 0; }
  if (a == 2) { r.push_back(4); a = 0; }
  if (a == 1) { r.push_back(2); a = 0; }
  while (m % 3 == 0) { r.push_back(3); m /= 3; }
  while (m % 5 == 0) { r.push_back(5); m /= 5; }
  if (m != 1 || (int)r.size() > ns::kMaxStages) return false;
  if (radices) *radices = r;
  return true;
}

bool cube_family_host(int mask) { return mask == NS_MASK_CUBE || mask == NS_MASK_ROGALLO; }

bool retained_host(const Geom& g, long long kx, long long ky, long long kz) {
  if (cube_family_host(g.mask)) {
    if (std::llabs(kx) > g.kmax || std::llabs(ky) > g.kmax || kz > g.kmax) return false;
  } else if (kx * kx + ky * ky + kz * kz > g.k2max) {
    return false;
  }
  if (g.mask < 2) return true;
  const long long a = std::llabs(kx), b = std::llabs(ky), c = std::llabs(kz), n2 = 2LL * g.n;
  return 3 * (a + b) < n2 && 3 * (a + c) < n2 && 3 * (b + c) < n2;
}

int kval_host(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

int isqrt_host(long long v) {
  if (v < 0) return -1;
  long long r = (long long)std::sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return (int)r;
}

int ybound_host(const Geom& g, int kz) {
  if (!cube_family_host(g.mask)) return isqrt_host(g.k2max - (long long)kz * kz);
  return kz <= g.kmax ? g.kmax : -1;
}

int num_shells(int n) {
  const long long k2top = 3LL * (n / 2) * (n / 2);
  const int r = isqrt_host(k2top);
  const int s = ((long long)r * (r + 1) >= k2top) ? r : r + 1;
  return s + 1;
}

const char* validate(const ns_config* c) {
  if (c == nullptr) return "config is NULL";
  if (!factor_ok(c->n, nullptr)) return "n must be 2^a 3^b 5^c with a >= 1 and 8 <= n <= 1024";
  if (c->precision != NS_FP32 && c->precision != NS_FP64) return "precision must be NS_FP32 or NS_FP64";
  if (c->mask < NS_MASK_SPHERE || c->mask > NS_MASK_ROGALLO)
    return "mask must be NS_MASK_SPHERE, NS_MASK_CUBE, NS_MASK_NO_MULTIPLE_ALIASES or NS_MASK_ROGALLO";
  if (c->flags & ~NS_CFG_GENERIC_PASSES) return "unknown config flags";
  if (!(c->nu >= 0.0) || !std::isfinite(c->nu)) return "nu must be finite and >= 0";
  if (!(c->ct > 0.0 && c->ct <= 1.0)) return "ct must satisfy 0 < ct <= 1";
  const double kmax = c->ct * c->n / 2.0;
  if (!cube_family_host(c->mask) ? largest_int_below(kmax * kmax) < 1 : largest_int_below(kmax) < 1)
    return "ct too small: no non-zero mode is retained";
  return nullptr;
}

// Sizes with specialised FP32 passes (ns_fast.hpp), unless the config asks for the
// size-generic ones.
bool fast_size(const ns_config* c) {
  const int n = c->n;
  return c->precision == NS_FP32 && !(c->flags & NS_CFG_GENERIC_PASSES) &&
         (n == 64 || n == 128 || n == 144 || n == 160 || n == 192 || n == 216 || n == 240 || n == 256 ||
          n == 270 || n == 324 || n == 360 || n == 384 || n == 512);
}

bool make_layout(const ns_config* c, Layout* lay) {
  std::vector<int> rad;
  factor_ok(c->n, &rad);
  Geom& g = lay->g;
  const int n = c->n;
  g.n = n;
  g.h = n / 2 + 1;
  g.mask = c->mask;
  const double kmax = c->ct * n / 2.0;
  if (!cube_family_host(c->mask)) {
    g.k2max = largest_int_below(kmax * kmax);
    g.kmax = isqrt_host(g.k2max);
    lay->k2top = g.k2max;
  } else {
    g.kmax = (int)largest_int_below(kmax);
    g.k2max = 3LL * g.kmax * g.kmax;
    lay->k2top = g.k2max;
  }
  g.kzn = g.kmax + 1;
  lay->elem = c->precision == NS_FP32 ? 8 : 16;
  int L = c->precision == NS_FP32 ? 16 : 8;
  int tx = 0;
  for (;;) {
    tx = (n * L + kEpt - 1) / kEpt;
    tx = (tx + 63) / 64 * 64;
    // the specialised passes always tile 16 columns (the generic kernels, which
    // would need more than 512 threads for that at N > 256, are not used then)
    if (tx <= 512 || L == 1 || fast_size(c)) break;
    L /= 2;
  }
  g.L = L;
  g.lgL = 0;
  while ((1 << g.lgL) < L) ++g.lgL;
  lay->tx = tx;
  g.kzp = (g.kzn + L - 1) / L * L;
  g.comp = (long long)n * n * g.h;
  g.wcomp = (long long)n * n * g.kzp;
  lay->ntz = (g.kzn + L - 1) / L;
  lay->ntzf = (g.h + L - 1) / L;
  // z pass: P lines per block, P a power of two dividing n^2, 3 P n <= kEptZ * tz
  int pz = 2;
  while (3 * (2 * pz) * n <= kEptZ * 256 && ((long long)n * n) % (2 * pz) == 0 && 2 * pz <= 32) pz *= 2;
  int tz = 256;
  while (3 * pz * n > kEptZ * tz) tz *= 2;
  lay->pz = pz;
  lay->tz = tz;
  int pa = pz;
  while (pa > 2 && 9 * pa * n > 2 * kEptZ * 512) pa /= 2;
  int ta = 256;
  while (9 * pa * n > 2 * kEptZ * ta) ta *= 2;
  lay->pa = (ta <= 512) ? pa : 0;
  lay->ta = ta;
  // plan
  FftPlan& p = lay->plan;
  std::memset(&p, 0, sizeof(p));
  p.n = n;
  p.nstages = (int)rad.size();
  int ns = 1;
  for (int s = 0; s < p.nstages; ++s) {
    p.radix[s] = rad[s];
    p.ns[s] = ns;
    p.tstride[s] = n / (ns * rad[s]);
    ns *= rad[s];
  }
  // active (k_y, k_z tile) lines of the x passes
  lay->tiles.clear();
  for (int yi = 0; yi < n; ++yi) {
    const int ky = kval_host(yi, n);
    for (int t = 0; t < lay->ntz; ++t) {
      const int kz0 = t * L;
      if (kz0 < g.kzn && std::abs(ky) <= ybound_host(g, kz0)) lay->tiles.push_back(make_int2(yi, kz0));
    }
  }
  lay->ntiles_active = (int)lay->tiles.size();
  lay->nsh = num_shells(n);
  lay->nbins = 3 * lay->nsh + 3 * g.h + 5;
  // workspace
  const size_t e = lay->elem, rsz = e / 2;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, kAlign); return o; };
  lay->off_tw = take(n * e);
  lay->off_etab = take(2 * (size_t)(lay->k2top + 1) * rsz);
  lay->off_force = take(3 * 196 * e);
  lay->off_tiles = take(lay->tiles.size() * sizeof(int2) + 8);
  lay->off_w = take(9 * (size_t)g.wcomp * e);
  lay->off_s = take(3 * (size_t)g.wcomp * e);   // stage buffers in the compact layout
  lay->off_a = take(3 * (size_t)g.wcomp * e);
  lay->off_spec = take((size_t)kSpecBlocks * lay->nbins * sizeof(double));
  lay->off_specout = take((size_t)lay->nbins * sizeof(double));
  lay->off_fstate = take(sizeof(ns::ForceState));
  lay->off_budget = take(sizeof(ns::Budget));
  lay->off_bpart = take(2 * (size_t)ns::kBudgetBlocks * sizeof(double));
  lay->total = off;
  return true;
}

// One evaluation of the nonlinear term on `in` (layout lin) with the shift s (NULL
// or all zero = unshifted); the x-forward epilogue applies OP with the operands
// and layouts in a.
template <typename R, int OP>
ns_status eval(ns_ctx* c, const Cx<R>* in, ns::Lay lin, const double* s, EpiArgs<R> a, Chain* ch = nullptr) {
  const Layout& l = c->lay;
  const Geom& g = l.g;
  Ptrs<R> p = ptrs<R>(c);
  const ns::Shift sh = make_shift(s);
  hipError_t e;
  if constexpr (std::is_same<R, float>::value) {
    switch (c->fast) {
      case 64: return fast_eval<64, OP>(c, in, lin, sh, a, ch);
      case 128: return fast_eval<128, OP>(c, in, lin, sh, a, ch);
      case 144: return fast_eval<144, OP>(c, in, lin, sh, a, ch);
      case 160: return fast_eval<160, OP>(c, in, lin, sh, a, ch);
      case 192: return fast_eval<192, OP>(c, in, lin, sh, a, ch);
      case 216: return fast_eval<216, OP>(c, in, lin, sh, a, ch);
      case 240: return fast_eval<240, OP>(c, in, lin, sh, a, ch);
      case 256: return fast_eval<256, OP>(c, in, lin, sh, a, ch);
      case 270: return fast_eval<270, OP>(c, in, lin, sh, a, ch);
      case 324: return fast_eval<324, OP>(c, in, lin, sh, a, ch);
      case 360: return fast_eval<360, OP>(c, in, lin, sh, a, ch);
      case 384: return fast_eval<384, OP>(c, in, lin, sh, a, ch);
      case 512: return fast_eval<512, OP>(c, in, lin, sh, a, ch);
      default: break;
    }
  }
  if (ch) ch->fused = false;  // the size-generic passes run every x-inverse pass on its own
  const size_t lds = lds_strided(l);
  const int ntiles = l.ntiles_active;
  if (ntiles > 0) {
    auto k1 = ns::k_xinv<R, kEpt>;
    if ((e = allow_lds(k1, lds)) != hipSuccess) return hip_check(c, e, "k_xinv attribute");
    if ((e = tstart(c, 0)) != hipSuccess) return hip_check(c, e, "timing event");
    hipLaunchKernelGGL(k1, dim3(ntiles), dim3(l.tx), lds, c->stream, in, lin, p.W, p.tw, sh, p.tiles, g, l.plan);
    if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
    auto k2 = ns::k_ypass<R, kEpt, +1>;
    if ((e = allow_lds(k2, lds)) != hipSuccess) return hip_check(c, e, "k_ypass attribute");
    if ((e = tstart(c, 1)) != hipSuccess) return hip_check(c, e, "timing event");
    hipLaunchKernelGGL(k2, dim3(6 * g.n * l.ntz), dim3(l.tx), lds, c->stream, p.W, p.tw, 0, l.ntz, g,
                       l.plan);
    if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
    const size_t ldsz = lds_z(l);
    auto k3 = ns::k_zcross<R, kEptZ>;
    if ((e = allow_lds(k3, ldsz)) != hipSuccess) return hip_check(c, e, "k_zcross attribute");
    if ((e = tstart(c, 2)) != hipSuccess) return hip_check(c, e, "timing event");
    hipLaunchKernelGGL(k3, dim3((int)((long long)g.n * g.n / l.pz)), dim3(l.tz), ldsz, c->stream,
                       p.W, p.tw, l.pz, g, l.plan);
    if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
    auto k4 = ns::k_ypass<R, kEpt, -1>;
    if ((e = allow_lds(k4, lds)) != hipSuccess) return hip_check(c, e, "k_ypass attribute");
    if ((e = tstart(c, 3)) != hipSuccess) return hip_check(c, e, "timing event");
    hipLaunchKernelGGL(k4, dim3(3 * g.n * l.ntz), dim3(l.tx), lds, c->stream, p.W, p.tw, 0, l.ntz, g,
                       l.plan);
    if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
  }
  if ((e = tstart(c, 4)) != hipSuccess) return hip_check(c, e, "timing event");
  if ((e = launch_xfwd<R, OP>(c, p, sh, a)) != hipSuccess) return hip_check(c, e, "k_xfwd launch");
  if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
  return hip_check(c, hipGetLastError(), "nonlinear-term launch");
}

// Epilogue operands; every layout defaults to the compact internal one.
template <typename R>
EpiArgs<R> epi(ns_ctx* c, int full) {
  EpiArgs<R> a;
  std::memset(&a, 0, sizeof(a));
  Ptrs<R> p = ptrs<R>(c);
  a.eh = p.eh;
  a.edt = p.edt;
  a.full = full;
  a.w = R(0.5);
  a.ntzf = c->lay.ntzf;
  a.lo0 = a.lo1 = a.li0 = a.li1 = compact_lay(c->lay);
  return a;
}

template <typename R>
ns_status nonlinear_t(ns_ctx* c, const void* u, void* nh, const double* shift, int flags) {
  const Cx<R>* in = static_cast<const Cx<R>*>(u);
  Cx<R>* out = static_cast<Cx<R>*>(nh);
  const ns::Lay U = user_lay(c->lay);
  EpiArgs<R> a = epi<R>(c, 1);
  a.out0 = out;
  a.lo0 = a.li1 = U;
  if (flags & NS_NL_PS_AVG) {
    const double zero[3] = {0, 0, 0}, half[3] = {0.5, 0.5, 0.5};
    ns_status st = eval<R, ns::OP_STORE>(c, in, U, zero, a);
    if (st != NS_OK) return st;
    a.in1 = out;
    return eval<R, ns::OP_AVG>(c, in, U, half, a);
  }
  return eval<R, ns::OP_STORE>(c, in, U, shift, a);
}

// exp(-nu k^2 dt/2) and exp(-nu k^2 dt) tables; kept while dt does not change.
template <typename R>
ns_status etab(ns_ctx* c, double dt) {
  if (c->etab_dt == dt) return NS_OK;
  Ptrs<R> p = ptrs<R>(c);
  const long long nt = c->lay.k2top + 1;
  hipLaunchKernelGGL(ns::k_etab<R>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream, p.eh,
                     p.edt, c->lay.k2top, c->cfg.nu, dt);
  ns_status st = hip_check(c, hipGetLastError(), "k_etab launch");
  if (st == NS_OK) c->etab_dt = dt;
  return st;
}

// Draw the forcing of step `step` from the state x (layout lx) into the workspace
// table and the FP64 forcing record.
template <typename R>
ns_status forcing_draw(ns_ctx* c, const Cx<R>* x, ns::Lay lx, const ns_forcing* fo, long long step, double dt) {
  Ptrs<R> p = ptrs<R>(c);
  hipLaunchKernelGGL(ns::k_forcing<R>, dim3(1), dim3(192), 0, c->stream, x, p.force, p.fstate, c->lay.g.n, lx.pitch,
                     lx.cs, fo->seed, step, dt, fo->injection);
  return hip_check(c, hipGetLastError(), "k_forcing launch");
}

// Energy-budget update from the state y (layout ly) after a step of length dt
// (dt = 0: start the budget at y); no-op while the budget is off.
template <typename R>
ns_status budget_sample(ns_ctx* c, const Cx<R>* y, ns::Lay ly, double dt, bool forced) {
  if (!c->budget) return NS_OK;
  Ptrs<R> p = ptrs<R>(c);
  hipLaunchKernelGGL(ns::k_budget_partial<R>, dim3(ns::kBudgetBlocks), dim3(256), 0, c->stream, y, ly, c->lay.g,
                     c->cfg.nu, p.bpart);
  hipLaunchKernelGGL(ns::k_budget_step, dim3(1), dim3(64), 0, c->stream, p.bpart, ns::kBudgetBlocks, p.budget,
                     p.fstate, dt, forced ? 1 : 0);
  return hip_check(c, hipGetLastError(), "budget launch");
}

template <typename R>
ns_status rk4_t(ns_ctx* c, void* u, double dt, int nsteps, const ns_forcing* fo, long long step0) {
  Cx<R>* s0 = static_cast<Cx<R>*>(u);
  Ptrs<R> p = ptrs<R>(c);
  const ns::Lay U = user_lay(c->lay), K = compact_lay(c->lay);
  ns_status st = etab<R>(c, dt);
  if (st != NS_OK) return st;
  // Between the steps of one call the state stays in scratch fields 6..8 (compact
  // rows, retained modes only; the forward passes use fields 0..5): the first step
  // reads the caller's array, the last writes it back whole.
  // Each x-forward pass also runs the next evaluation's x-inverse pass on the stage
  // state it computes (Chain), except after the last step.
  Cx<R>* xs = p.W + 6 * c->lay.g.wcomp;
  bool fused = false;
  for (int i = 0; i < nsteps; ++i) {
    const bool first = (i == 0), last = (i == nsteps - 1);
    Cx<R>* x = first ? s0 : xs;
    const ns::Lay lx = first ? U : K;
    EpiArgs<R> a = epi<R>(c, 0);
    a.dt = R(dt);
    a.in0 = x;
    a.li0 = lx;
    a.in1 = p.ab;
    a.out0 = p.ab;
    a.out1 = p.sb;
    if (fo != nullptr) {
      // the forcing of this step, drawn from its start state, enters all four slopes
      if ((st = forcing_draw<R>(c, x, lx, fo, step0 + i, dt)) != NS_OK) return st;
      a.force = p.force;
    }
    Chain ch;
    ch.feed = 2;
    ch.front_done = fused;
    if ((st = eval<R, ns::OP_RK4_0>(c, x, lx, nullptr, a, &ch)) != NS_OK) return st;
    ch.front_done = ch.fused;
    if ((st = eval<R, ns::OP_RK4_1>(c, p.sb, K, nullptr, a, &ch)) != NS_OK) return st;
    ch.front_done = ch.fused;
    if ((st = eval<R, ns::OP_RK4_2>(c, p.sb, K, nullptr, a, &ch)) != NS_OK) return st;
    EpiArgs<R> f = epi<R>(c, last ? 1 : 0);
    f.dt = R(dt);
    f.in1 = p.ab;
    f.out0 = last ? s0 : xs;
    f.lo0 = last ? U : K;
    f.force = a.force;
    ch.front_done = ch.fused;
    ch.feed = last ? 0 : 1;
    if ((st = eval<R, ns::OP_RK4_3>(c, p.sb, K, nullptr, f, &ch)) != NS_OK) return st;
    fused = ch.fused;
    if ((st = budget_sample<R>(c, last ? s0 : xs, last ? U : K, dt, fo != nullptr)) != NS_OK) return st;
  }
  return NS_OK;
}

uint64_t sm64_mix_host(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double sm64_uniform_host(uint64_t seed, long long step, long long j) {
  const uint64_t G = 0x9E3779B97F4A7C15ull;
  const uint64_t s = sm64_mix_host(seed + G * (uint64_t)(step + 1));
  return (double)(sm64_mix_host(s + G * (uint64_t)(j + 1)) >> 11) * (1.0 / 9007199254740992.0);
}

template <typename R>
ns_status ps_t(ns_ctx* c, void* u, double dt, int nsteps, int variant, const double* alphas,
               const ns_forcing* fo, long long step0, void* stage1) {
  Cx<R>* s0 = static_cast<Cx<R>*>(u);
  Ptrs<R> p = ptrs<R>(c);
  const ns::Lay U = user_lay(c->lay), K = compact_lay(c->lay);
  ns_status st = etab<R>(c, dt);
  if (st != NS_OK) return st;
  const double zero[3] = {0, 0, 0}, half[3] = {0.5, 0.5, 0.5};
  // Between the steps of one call the state stays in scratch fields 6..8 (compact
  // rows, retained modes only; the forward passes use fields 0..5): the first step
  // reads the caller's array (x), the last writes it back whole (y).
  Cx<R>* xs = p.W + 6 * c->lay.g.wcomp;
  bool fused = false;  // the next evaluation's x-inverse pass already ran
  // one step; the state after it is in y (layout ly)
  auto step = [&](int i) -> ns_status {
    ns_status st;
    const bool first = (i == 0), last = (i == nsteps - 1);
    Cx<R>* x = first ? s0 : xs;
    Cx<R>* y = last ? s0 : xs;
    const ns::Lay lx = first ? U : K, ly = last ? U : K;
    const int fy = last ? 1 : 0;
    if (variant == NS_RK2) {
      // midpoint RK2 without shifts: S_h = E_h (S0 + dt/2 N(S0)); S = E_dt S0 + dt E_h N(S_h)
      EpiArgs<R> a = epi<R>(c, 0);
      a.dt = R(dt);
      a.in0 = x;
      a.li0 = lx;
      a.out0 = p.sb;
      if ((st = eval<R, ns::OP_MID1>(c, x, lx, zero, a)) != NS_OK) return st;
      EpiArgs<R> f = epi<R>(c, fy);
      f.dt = R(dt);
      f.in0 = x;
      f.li0 = lx;
      f.out0 = y;
      f.lo0 = ly;
      if ((st = eval<R, ns::OP_MID2>(c, p.sb, K, zero, f)) != NS_OK) return st;
      return NS_OK;
    }
    if (variant == NS_EULER || variant == NS_EULER_PS) {
      // S = E_dt (S0 + dt N_a) with N_a = N(S0) or the two-shift average
      EpiArgs<R> f = epi<R>(c, fy);
      f.dt = R(dt);
      f.in0 = x;
      f.li0 = lx;
      f.out0 = y;
      f.lo0 = ly;
      if (variant == NS_EULER) {
        if ((st = eval<R, ns::OP_EUL>(c, x, lx, zero, f)) != NS_OK) return st;
        return NS_OK;
      }
      EpiArgs<R> a = epi<R>(c, 0);
      a.out0 = p.ab;
      if ((st = eval<R, ns::OP_STORE>(c, x, lx, zero, a)) != NS_OK) return st;
      f.in1 = p.ab;
      if ((st = eval<R, ns::OP_EULAV>(c, x, lx, half, f)) != NS_OK) return st;
      return NS_OK;
    }
    if (variant == NS_PS_EXACT || variant == NS_PS_EXACT8) {
      // midpoint RK2 with every evaluation the average over ns shifts: the first
      // ns - 1 are summed into ab, the last closes the stage with weight w = 1/ns
      // (ns = 2: shifts 0 and (1/2,1/2,1/2); ns = 8: the shifts in {0, 1/2}^3)
      const double s2[2][3] = {{0, 0, 0}, {0.5, 0.5, 0.5}};
      const double s8[8][3] = {{0, 0, 0},     {0, 0, 0.5},   {0, 0.5, 0},   {0, 0.5, 0.5},
                               {0.5, 0, 0},   {0.5, 0, 0.5}, {0.5, 0.5, 0}, {0.5, 0.5, 0.5}};
      const int ns = variant == NS_PS_EXACT ? 2 : 8;
      const double(*sh)[3] = variant == NS_PS_EXACT ? s2 : s8;
      for (int stage = 0; stage < 2; ++stage) {
        const Cx<R>* z = stage == 0 ? x : p.sb;
        const ns::Lay lz = stage == 0 ? lx : K;
        EpiArgs<R> a = epi<R>(c, 0);
        a.out0 = p.ab;
        // the first evaluation of a stage may already have its x-inverse pass, run by
        // the x-forward pass that computed its state
        Chain c0;
        c0.front_done = fused;
        if ((st = eval<R, ns::OP_STORE>(c, z, lz, sh[0], a, &c0)) != NS_OK) return st;
        a.in1 = p.ab;
        for (int j = 1; j < ns - 1; ++j)
          if ((st = eval<R, ns::OP_ACC>(c, z, lz, sh[j], a)) != NS_OK) return st;
        EpiArgs<R> f = epi<R>(c, stage == 0 ? 0 : fy);
        f.dt = R(dt);
        f.w = R(1.0 / ns);
        f.in0 = x;
        f.li0 = lx;
        f.in1 = p.ab;
        Chain ch;
        ch.feed = (stage == 0 || !last) ? 1 : 0;
        ch.next_s = sh[0];
        if (stage == 0) {
          f.out0 = p.sb;
          if ((st = eval<R, ns::OP_EX1B>(c, z, lz, sh[ns - 1], f, &ch)) != NS_OK) return st;
        } else {
          f.out0 = y;
          f.lo0 = ly;
          if ((st = eval<R, ns::OP_EX2B>(c, z, lz, sh[ns - 1], f, &ch)) != NS_OK) return st;
        }
        fused = ch.fused;
      }
      return NS_OK;
    }
    // Heun: the first-stage shifts of this step and of the next (the x-forward pass
    // of the second stage runs the next step's first x-inverse pass)
    double al[3] = {0, 0, 0}, an[3] = {0, 0, 0};
    if (variant == NS_PS_RANDOM) {
      for (int j = 0; j < 3; ++j) {
        al[j] = alphas ? alphas[3 * i + j] : sm64_uniform_host(c->cfg.seed, step0 + i, j);
        if (!last) an[j] = alphas ? alphas[3 * (i + 1) + j] : sm64_uniform_host(c->cfg.seed, step0 + i + 1, j);
      }
    }
    double be[3];
    for (int j = 0; j < 3; ++j) be[j] = std::fmod(al[j] + 0.5, 1.0);
    EpiArgs<R> a = epi<R>(c, 0);
    a.dt = R(dt);
    a.in0 = x;
    a.li0 = lx;
    a.out0 = p.ab;
    a.out1 = p.sb;
    // with stage1 the first-stage state is written to the caller's array (state
    // layout, retained modes) and read back from there, not fed through registers
    Cx<R>* s1 = stage1 ? static_cast<Cx<R>*>(stage1) : p.sb;
    const ns::Lay l1 = stage1 ? U : K;
    if (stage1) {
      a.out1 = s1;
      a.lo1 = U;
    }
    if (fo != nullptr) {
      if ((st = forcing_draw<R>(c, x, lx, fo, step0 + i, dt)) != NS_OK) return st;
      a.force = p.force;
    }
    Chain ch;
    ch.front_done = fused;
    ch.feed = stage1 ? 0 : 2;
    ch.next_s = be;
    if ((st = eval<R, ns::OP_HEUN1>(c, x, lx, al, a, &ch)) != NS_OK) return st;
    EpiArgs<R> f = epi<R>(c, fy);
    f.dt = R(dt);
    f.in1 = p.ab;
    f.out0 = y;
    f.lo0 = ly;
    ch.front_done = ch.fused;
    ch.feed = last ? 0 : 1;
    ch.next_s = an;
    if ((st = eval<R, ns::OP_HEUN2>(c, s1, l1, be, f, &ch)) != NS_OK) return st;
    fused = ch.fused;
    return NS_OK;
  };
  for (int i = 0; i < nsteps; ++i) {
    const bool last = (i == nsteps - 1);
    if ((st = step(i)) != NS_OK) return st;
    if ((st = budget_sample<R>(c, last ? s0 : xs, last ? U : K, dt, fo != nullptr)) != NS_OK) return st;
  }
  return NS_OK;
}


// One transposed linearised evaluation at state `st` (layout lst) with shift s:
// lam-pass input from `la`, adjoint stage combination AOP in the last pass.
template <typename R, int AOP>
ns_status adj_eval(ns_ctx* c, const Cx<R>* st, ns::Lay lst, const double* s, const LamArgs<R>& la,
                   AdjArgs<R> aa) {
  const Layout& l = c->lay;
  const Geom& g = l.g;
  Ptrs<R> p = ptrs<R>(c);
  const ns::Shift sh = make_shift(s);
  hipError_t e;
  if constexpr (std::is_same<R, float>::value) {
    switch (c->fast) {
      case 64: return fast_adj_eval<64, AOP>(c, st, lst, sh, la, aa);
      case 128: return fast_adj_eval<128, AOP>(c, st, lst, sh, la, aa);
      case 144: return fast_adj_eval<144, AOP>(c, st, lst, sh, la, aa);
      case 160: return fast_adj_eval<160, AOP>(c, st, lst, sh, la, aa);
      case 192: return fast_adj_eval<192, AOP>(c, st, lst, sh, la, aa);
      case 216: return fast_adj_eval<216, AOP>(c, st, lst, sh, la, aa);
      case 240: return fast_adj_eval<240, AOP>(c, st, lst, sh, la, aa);
      case 256: return fast_adj_eval<256, AOP>(c, st, lst, sh, la, aa);
      case 270: return fast_adj_eval<270, AOP>(c, st, lst, sh, la, aa);
      case 324: return fast_adj_eval<324, AOP>(c, st, lst, sh, la, aa);
      case 360: return fast_adj_eval<360, AOP>(c, st, lst, sh, la, aa);
      case 384: return fast_adj_eval<384, AOP>(c, st, lst, sh, la, aa);
      case 512: return fast_adj_eval<512, AOP>(c, st, lst, sh, la, aa);
      default: break;
    }
  }
  const size_t lds = lds_strided(l);
  const int ntiles = l.ntiles_active;
  if (ntiles > 0) {
    auto k1 = ns::k_xinv<R, kEpt>;
    if ((e = allow_lds(k1, lds)) != hipSuccess) return hip_check(c, e, "k_xinv attribute");
    hipLaunchKernelGGL(k1, dim3(ntiles), dim3(l.tx), lds, c->stream, st, lst, p.W, p.tw, sh, p.tiles, g, l.plan);
    auto kl = ns::k_xlam<R, kEpt>;
    if ((e = allow_lds(kl, lds)) != hipSuccess) return hip_check(c, e, "k_xlam attribute");
    hipLaunchKernelGGL(kl, dim3(ntiles), dim3(l.tx), lds, c->stream, la, p.W, p.tw, sh, p.tiles, g, l.plan);
    auto k2 = ns::k_ypass<R, kEpt, +1>;
    if ((e = allow_lds(k2, lds)) != hipSuccess) return hip_check(c, e, "k_ypass attribute");
    hipLaunchKernelGGL(k2, dim3(9 * g.n * l.ntz), dim3(l.tx), lds, c->stream, p.W, p.tw, 0, l.ntz, g,
                       l.plan);
    const size_t ldsz = lds_zadj(l);
    auto k3 = ns::k_zadj<R, kEptZ>;
    if ((e = allow_lds(k3, ldsz)) != hipSuccess) return hip_check(c, e, "k_zadj attribute");
    hipLaunchKernelGGL(k3, dim3((int)((long long)g.n * g.n / l.pa)), dim3(l.ta), ldsz, c->stream,
                       p.W, p.tw, l.pa, g, l.plan);
    auto k4 = ns::k_ypass<R, kEpt, -1>;
    if ((e = allow_lds(k4, lds)) != hipSuccess) return hip_check(c, e, "k_ypass attribute");
    hipLaunchKernelGGL(k4, dim3(6 * g.n * l.ntz), dim3(l.tx), lds, c->stream, p.W, p.tw, 0, l.ntz, g,
                       l.plan);
  }
  auto k5 = ns::k_xadj<R, kEpt, AOP>;
  if ((e = allow_lds(k5, lds)) != hipSuccess) return hip_check(c, e, "k_xadj attribute");
  const int nblk = aa.full ? g.n * l.ntzf : ntiles;
  aa.ntzf = l.ntzf;
  if (nblk > 0)
    hipLaunchKernelGGL(k5, dim3(nblk), dim3(l.tx), lds, c->stream, p.W, p.tw, sh, p.tiles, g, l.plan, aa);
  return hip_check(c, hipGetLastError(), "adjoint launch");
}

template <typename R>
ns_status vjp_t(ns_ctx* c, const void* u0v, void* lamv, double dt, int variant, const double* alpha,
                const ns_forcing* fo, long long step, const void* stage1) {
  const Cx<R>* u0 = static_cast<const Cx<R>*>(u0v);
  Cx<R>* lam = static_cast<Cx<R>*>(lamv);
  Ptrs<R> p = ptrs<R>(c);
  const ns::Lay U = user_lay(c->lay), K = compact_lay(c->lay);
  ns_status st = etab<R>(c, dt);
  if (st != NS_OK) return st;
  const R rdt = R(dt);
  auto adj = [&](int full) {
    AdjArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.eh = p.eh;
    a.edt = p.edt;
    a.full = full;
    a.lo0 = a.li0 = a.li1 = K;
    return a;
  };
  auto lamargs = [&](const Cx<R>* A, ns::Lay LA, R cA, const R* eA, const Cx<R>* B, R cB, const R* eB) {
    LamArgs<R> la;
    la.A = A; la.B = B; la.eA = eA; la.eB = eB; la.cA = cA; la.cB = cB;
    la.la = LA;
    la.lb = K;
    return la;
  };
  const double zero[3] = {0, 0, 0}, half[3] = {0.5, 0.5, 0.5};
  if (variant == NS_PS_EXACT) {
    EpiArgs<R> f = epi<R>(c, 0);
    f.dt = rdt;
    f.out0 = p.ab;
    if ((st = eval<R, ns::OP_STORE>(c, u0, U, zero, f)) != NS_OK) return st;
    f.in0 = u0;
    f.li0 = U;
    f.in1 = p.ab;
    f.out0 = p.sb;
    if ((st = eval<R, ns::OP_EX1B>(c, u0, U, half, f)) != NS_OK) return st;  // sb = S_h
    LamArgs<R> l1 = lamargs(lam, U, R(0.5) * rdt, p.eh, nullptr, R(0), nullptr);
    AdjArgs<R> a = adj(0);
    a.out0 = p.ab;
    if ((st = adj_eval<R, ns::AOP_STORE>(c, p.sb, K, zero, l1, a)) != NS_OK) return st;
    a.in1 = p.ab;
    if ((st = adj_eval<R, ns::AOP_ACC>(c, p.sb, K, half, l1, a)) != NS_OK) return st;  // ab = mu
    LamArgs<R> l2 = lamargs(p.ab, K, R(0.25) * rdt, p.eh, nullptr, R(0), nullptr);
    a.in0 = lam;
    a.li0 = U;
    a.in1 = p.ab;
    a.out0 = lam;
    a.lo0 = U;
    if ((st = adj_eval<R, ns::AOP_EXACT>(c, u0, U, zero, l2, a)) != NS_OK) return st;
    AdjArgs<R> b = adj(1);
    b.in1 = lam;
    b.li1 = U;
    b.out0 = lam;
    b.lo0 = U;
    return adj_eval<R, ns::AOP_ACC>(c, u0, U, half, l2, b);
  }
  double al[3] = {0, 0, 0};
  if (variant == NS_PS_RANDOM)
    for (int j = 0; j < 3; ++j) al[j] = alpha[j];
  double be[3];
  for (int j = 0; j < 3; ++j) be[j] = std::fmod(al[j] + 0.5, 1.0);
  EpiArgs<R> f = epi<R>(c, 0);
  f.dt = rdt;
  f.in0 = u0;
  f.li0 = U;
  f.out0 = p.ab;
  f.out1 = p.sb;
  if (fo != nullptr) {
    // the forward step's forcing, redrawn from u0 (the draw is counter-based)
    if ((st = forcing_draw<R>(c, u0, U, fo, step, dt)) != NS_OK) return st;
    f.force = p.force;
  }
  // S1, the state the second stage is linearised at: the caller's (from the forward
  // step) or recomputed here
  const Cx<R>* s1 = p.sb;
  ns::Lay l1s = K;
  if (stage1 != nullptr) {
    s1 = static_cast<const Cx<R>*>(stage1);
    l1s = U;
  } else if ((st = eval<R, ns::OP_HEUN1>(c, u0, U, al, f)) != NS_OK) {
    return st;  // sb = S1
  }
  LamArgs<R> l1 = lamargs(lam, U, R(0.5) * rdt, p.eh, nullptr, R(0), nullptr);
  AdjArgs<R> a = adj(0);
  a.out0 = p.ab;
  if ((st = adj_eval<R, ns::AOP_STORE>(c, s1, l1s, be, l1, a)) != NS_OK) return st;  // ab = mu1
  const Geom& g = c->lay.g;
  if (fo != nullptr) {
    // the amplitude's dependence on u0: (da/dB) <mu_O, g>, formed while lam is still the input
    hipLaunchKernelGGL(ns::k_forcing_adj_dot<R>, dim3(1), dim3(64), 0, c->stream, lam, U, p.ab, K, p.eh, p.edt,
                       p.fstate, g.n, dt);
    if ((st = hip_check(c, hipGetLastError(), "k_forcing_adj_dot launch")) != NS_OK) return st;
  }
  LamArgs<R> l2 = lamargs(lam, U, R(0.5) * rdt, p.eh, p.ab, rdt, p.edt);
  AdjArgs<R> b = adj(1);
  b.in0 = lam;
  b.li0 = U;
  b.in1 = p.ab;
  b.out0 = lam;
  b.lo0 = U;
  if ((st = adj_eval<R, ns::AOP_HEUN>(c, u0, U, al, l2, b)) != NS_OK) return st;
  if (fo != nullptr) {
    hipLaunchKernelGGL(ns::k_forcing_adj_add<R>, dim3(1), dim3(64), 0, c->stream, lam, U, p.fstate, g.n);
    if ((st = hip_check(c, hipGetLastError(), "k_forcing_adj_add launch")) != NS_OK) return st;
  }
  return NS_OK;
}

// Enqueue the reduction and its copy into pinned host memory, then record an
// event: the result can be waited for without waiting for later work.
template <typename R>
ns_status spectra_enqueue_t(ns_ctx* c, const void* u, const void* nh) {
  const Layout& l = c->lay;
  Ptrs<R> p = ptrs<R>(c);
  ns_status st;
  if (c->pin_spec == nullptr) {
    void* h = nullptr;
    if ((st = hip_check(c, hipHostMalloc(&h, (size_t)l.nbins * sizeof(double), hipHostMallocDefault),
                        "pinned spectra buffer")) != NS_OK)
      return st;
    c->pin_spec = static_cast<double*>(h);
  }
  if (c->spec_ev == nullptr &&
      (st = hip_check(c, hipEventCreateWithFlags(&c->spec_ev, hipEventDisableTiming), "spectra event")) != NS_OK)
    return st;
  // wavefronts per block: up to 16, as many private bin sets as fit in 128 KB of LDS
  const size_t set = (size_t)l.nbins * sizeof(double);
  const int nwb = (int)std::max<size_t>(1, std::min<size_t>(16, (size_t)(128 * 1024) / set));
  const size_t lds = nwb * set;
  hipError_t e = allow_lds(ns::k_spectra<R>, lds);
  if (e != hipSuccess) return hip_check(c, e, "k_spectra attribute");
  hipLaunchKernelGGL(ns::k_spectra<R>, dim3(kSpecBlocks), dim3(64 * nwb), lds, c->stream,
                     static_cast<const Cx<R>*>(u), static_cast<const Cx<R>*>(nh), c->cfg.nu, l.g.n,
                     l.g.h, l.nsh, l.g.comp, p.spec);
  hipLaunchKernelGGL(ns::k_spectra_sum, dim3((l.nbins + 7) / 8), dim3(256), 0, c->stream, p.spec,
                     kSpecBlocks, l.nbins, p.specout);
  if ((st = hip_check(c, hipGetLastError(), "spectra launch")) != NS_OK) return st;
  if ((st = hip_check(c, hipMemcpyAsync(c->pin_spec, p.specout, l.nbins * sizeof(double),
                                        hipMemcpyDeviceToHost, c->stream), "spectra copy")) != NS_OK)
    return st;
  if ((st = hip_check(c, hipEventRecord(c->spec_ev, c->stream), "spectra event record")) != NS_OK) return st;
  c->spec_pending = true;
  return NS_OK;
}

ns_status spectra_wait(ns_ctx* c, ns_spectra_out* out) {
  if (!c->spec_pending) return fail(c, NS_ERR_STATE, "no spectra reduction in flight");
  ns_status st = hip_check(c, hipEventSynchronize(c->spec_ev), "spectra wait");
  if (st != NS_OK) return st;
  c->spec_pending = false;
  const Layout& l = c->lay;
  const double* b = c->pin_spec;
  const int nsh = l.nsh, h = l.g.h;
  if (out->e_shell) std::memcpy(out->e_shell, b, nsh * sizeof(double));
  if (out->d_shell) std::memcpy(out->d_shell, b + nsh, nsh * sizeof(double));
  if (out->t_shell) std::memcpy(out->t_shell, b + 2 * nsh, nsh * sizeof(double));
  if (out->e_1d) std::memcpy(out->e_1d, b + 3 * nsh, 3 * h * sizeof(double));
  if (out->totals) std::memcpy(out->totals, b + 3 * nsh + 3 * h, 5 * sizeof(double));
  if (b[3 * nsh + 3 * h + 4] != 0.0) return fail(c, NS_ERR_NONFINITE, "non-finite entries in input");
  return NS_OK;
}

}  // namespace

namespace {

// Host checks of a forcing argument (NULL is valid: no forcing).
ns_status check_forcing(ns_ctx* ctx, const ns_forcing* forcing) {
  if (forcing == nullptr) return NS_OK;
  if (forcing->k2_lo != 4 || forcing->k2_hi != 9) return fail(ctx, NS_ERR_ARG, "forcing shell must be 4 <= |k|^2 <= 9");
  if (!(forcing->injection > 0.0) || !std::isfinite(forcing->injection))
    return fail(ctx, NS_ERR_ARG, "injection must be finite and > 0");
  const Geom& g = ctx->lay.g;
  for (int kx = -3; kx <= 3; ++kx)
    for (int ky = -3; ky <= 3; ++ky)
      for (int kz = 0; kz <= 3; ++kz) {
        const int k2 = kx * kx + ky * ky + kz * kz;
        if (k2 >= 4 && k2 <= 9 && !retained_host(g, kx, ky, kz))
          return fail(ctx, NS_ERR_ARG, "forcing shell lies outside the retained set");
      }
  return NS_OK;
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

size_t ns_workspace_bytes(const ns_config* cfg) {
  const char* m = validate(cfg);
  if (m) { g_last_error = m; return 0; }
  Layout lay;
  make_layout(cfg, &lay);
  return lay.total;
}

int32_t ns_num_shells(int32_t n) { return n >= 2 ? num_shells(n) : 0; }

int64_t ns_retained_bound(const ns_config* cfg) {
  const char* m = validate(cfg);
  if (m) { g_last_error = m; return -1; }
  Layout lay;
  make_layout(cfg, &lay);
  return !cube_family_host(cfg->mask) ? lay.g.k2max : lay.g.kmax;
}

ns_status ns_init(const ns_config* cfg, void* workspace, size_t ws_bytes, ns_ctx** out) {
  if (out == nullptr) return fail(nullptr, NS_ERR_ARG, "out is NULL");
  const char* m = validate(cfg);
  if (m) return fail(nullptr, NS_ERR_ARG, m);
  if (!aligned(workspace)) return fail(nullptr, NS_ERR_ARG, "workspace must be a non-NULL 256-byte aligned device pointer");
  ns_ctx* c = new (std::nothrow) ns_ctx;
  if (!c) return fail(nullptr, NS_ERR_STATE, "out of host memory");
  c->cfg = *cfg;
  c->stream = static_cast<hipStream_t>(cfg->stream);
  make_layout(cfg, &c->lay);
  if (ws_bytes < c->lay.total) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "workspace too small: %zu bytes given, %zu needed", ws_bytes, c->lay.total);
    delete c;
    return fail(nullptr, NS_ERR_SIZE, msg);
  }
  c->ws = static_cast<char*>(workspace);
  if (fast_size(cfg) && c->lay.g.L == ns::kFastL) c->fast = cfg->n;
  // twiddles W_N^t = exp(-2 pi i t/N), long double, rounded once
  const int n = cfg->n;
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<char> tw(n * c->lay.elem);
  for (int t = 0; t < n; ++t) {
    const long double a = -2.0L * pi * (long double)t / (long double)n;
    const long double cs = std::cos(a), sn = std::sin(a);
    if (cfg->precision == NS_FP32) {
      float v[2] = {(float)cs, (float)sn};
      std::memcpy(tw.data() + t * 8, v, 8);
    } else {
      double v[2] = {(double)cs, (double)sn};
      std::memcpy(tw.data() + t * 16, v, 16);
    }
  }
  hipError_t e = hipMemcpyAsync(c->ws + c->lay.off_tw, tw.data(), tw.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !c->lay.tiles.empty())
    e = hipMemcpyAsync(c->ws + c->lay.off_tiles, c->lay.tiles.data(), c->lay.tiles.size() * sizeof(int2),
                       hipMemcpyHostToDevice, c->stream);
  // the FP64 records start at zero (an empty budget, no forcing drawn yet)
  const std::vector<char> zero(sizeof(ns::ForceState) + sizeof(ns::Budget), 0);
  if (e == hipSuccess) {
    e = hipMemcpyAsync(c->ws + c->lay.off_fstate, zero.data(), sizeof(ns::ForceState), hipMemcpyHostToDevice,
                       c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->ws + c->lay.off_budget, zero.data(), sizeof(ns::Budget), hipMemcpyHostToDevice,
                         c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    std::string msg = std::string("upload of tables failed: ") + hipGetErrorString(e);
    delete c;
    return fail(nullptr, NS_ERR_HIP, msg);
  }
  *out = c;
  return NS_OK;
}

ns_status ns_destroy(ns_ctx* ctx) {
  delete ctx;
  return NS_OK;
}

const char* ns_last_error(const ns_ctx* ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }

ns_status ns_set_stream(ns_ctx* ctx, void* stream) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(stream);
  ctx->cfg.stream = stream;
  return NS_OK;
}

ns_status ns_nonlinear(ns_ctx* ctx, const void* u_hat, void* n_hat, const double shift[3], int32_t flags) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  if (!aligned(u_hat) || !aligned(n_hat)) return fail(ctx, NS_ERR_ARG, "u_hat and n_hat must be non-NULL 256-byte aligned device pointers");
  if (u_hat == n_hat) return fail(ctx, NS_ERR_ARG, "u_hat and n_hat must not overlap");
  if (flags & ~NS_NL_PS_AVG) return fail(ctx, NS_ERR_ARG, "unknown flags");
  if (shift && !(std::isfinite(shift[0]) && std::isfinite(shift[1]) && std::isfinite(shift[2])))
    return fail(ctx, NS_ERR_ARG, "shift must be finite");
  return ctx->cfg.precision == NS_FP32 ? nonlinear_t<float>(ctx, u_hat, n_hat, shift, flags)
                                       : nonlinear_t<double>(ctx, u_hat, n_hat, shift, flags);
}

ns_status ns_step_rk4_trunc(ns_ctx* ctx, void* u_hat, double dt, int32_t nsteps, const ns_forcing* forcing,
                            int64_t step0) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  if (!aligned(u_hat)) return fail(ctx, NS_ERR_ARG, "u_hat must be a non-NULL 256-byte aligned device pointer");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, NS_ERR_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(ctx, NS_ERR_ARG, "nsteps must be >= 0");
  ns_status st = check_forcing(ctx, forcing);
  if (st != NS_OK) return st;
  if (nsteps == 0) return NS_OK;
  return ctx->cfg.precision == NS_FP32 ? rk4_t<float>(ctx, u_hat, dt, nsteps, forcing, step0)
                                       : rk4_t<double>(ctx, u_hat, dt, nsteps, forcing, step0);
}

ns_status ns_step_rk2_phaseshift(ns_ctx* ctx, void* u_hat, double dt, int32_t nsteps, int32_t variant,
                                 const double* alphas, const ns_forcing* forcing, int64_t step0, void* stage1) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  if (!aligned(u_hat)) return fail(ctx, NS_ERR_ARG, "u_hat must be a non-NULL 256-byte aligned device pointer");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, NS_ERR_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(ctx, NS_ERR_ARG, "nsteps must be >= 0");
  if (variant < NS_PS_EXACT || variant > NS_PS_EXACT8) return fail(ctx, NS_ERR_ARG, "unknown scheme variant");
  if (forcing && variant != NS_PS_APPROX && variant != NS_PS_RANDOM)
    return fail(ctx, NS_ERR_ARG, "forcing is supported by the Heun variants only");
  ns_status fst = check_forcing(ctx, forcing);
  if (fst != NS_OK) return fst;
  if (alphas && variant == NS_PS_RANDOM)
    for (int i = 0; i < 3 * nsteps; ++i)
      if (!std::isfinite(alphas[i])) return fail(ctx, NS_ERR_ARG, "alphas must be finite");
  if (stage1 != nullptr) {
    if (variant != NS_PS_APPROX && variant != NS_PS_RANDOM)
      return fail(ctx, NS_ERR_ARG, "stage1 is kept by the Heun variants only");
    if (nsteps != 1) return fail(ctx, NS_ERR_ARG, "stage1 needs nsteps == 1");
    if (!aligned(stage1) || stage1 == u_hat)
      return fail(ctx, NS_ERR_ARG, "stage1 must be a 256-byte aligned device array distinct from u_hat");
  }
  if (nsteps == 0) return NS_OK;
  return ctx->cfg.precision == NS_FP32
             ? ps_t<float>(ctx, u_hat, dt, nsteps, variant, alphas, forcing, step0, stage1)
             : ps_t<double>(ctx, u_hat, dt, nsteps, variant, alphas, forcing, step0, stage1);
}

namespace {

// Host checks shared by the two entry points of the 1D model; the message is kept
// as the thread's last error.
ns_status check1d(int32_t n, double ct, int32_t batch, const void* a, const void* b, int* kmax) {
  if (n < 4 || n > 1024 || (n % 2) != 0) return fail(nullptr, NS_ERR_ARG, "n must be even with 4 <= n <= 1024");
  if (!(ct > 0.0 && ct <= 1.0)) return fail(nullptr, NS_ERR_ARG, "ct must satisfy 0 < ct <= 1");
  const long long km = largest_int_below(ct * n / 2.0);
  if (km < 1) return fail(nullptr, NS_ERR_ARG, "ct too small: no non-zero mode is retained");
  if (batch < 0) return fail(nullptr, NS_ERR_ARG, "batch must be >= 0");
  for (const void* p : {a, b})
    if (batch > 0 && (p == nullptr || (reinterpret_cast<uintptr_t>(p) % 16) != 0))
      return fail(nullptr, NS_ERR_ARG, "spectra must be non-NULL 16-byte aligned device pointers");
  *kmax = (int)km;
  return NS_OK;
}

ns_status launch1d(const ns1d::Args& a, int32_t batch, void* stream) {
  if (batch == 0) return NS_OK;
  const size_t lds = ns1d::lds_bytes(a.n);
  hipError_t e = allow_lds(ns1d::k_model1d, lds);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(ns1d::k_model1d, dim3((unsigned)batch), dim3(ns1d::kThreads), lds,
                       static_cast<hipStream_t>(stream), a);
    e = hipGetLastError();
  }
  return hip_check(nullptr, e, "1D model launch");
}

}  // namespace

ns_status ns1d_nonlinear(const void* s_hat, void* n_hat, int32_t n, double ct, int32_t batch, double shift,
                         void* stream) {
  int kmax = 0;
  ns_status st = check1d(n, ct, batch, s_hat, n_hat, &kmax);
  if (st != NS_OK) return st;
  if (!std::isfinite(shift)) return fail(nullptr, NS_ERR_ARG, "shift must be finite");
  ns1d::Args a{static_cast<const double2*>(s_hat), static_cast<double2*>(n_hat), n, n / 2 + 1, kmax, 0.0, 0, -1,
               shift};
  return launch1d(a, batch, stream);
}

ns_status ns1d_step(void* s_hat, int32_t n, double ct, int32_t batch, double dt, int32_t nsteps, int32_t scheme,
                    void* stream) {
  int kmax = 0;
  ns_status st = check1d(n, ct, batch, s_hat, s_hat, &kmax);
  if (st != NS_OK) return st;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(nullptr, NS_ERR_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(nullptr, NS_ERR_ARG, "nsteps must be >= 0");
  if (scheme < NS1D_EULER || scheme > NS1D_RK4) return fail(nullptr, NS_ERR_ARG, "unknown 1D scheme");
  if (nsteps == 0) return NS_OK;
  ns1d::Args a{static_cast<const double2*>(s_hat), static_cast<double2*>(s_hat), n, n / 2 + 1, kmax, dt, nsteps,
               scheme, 0.0};
  return launch1d(a, batch, stream);
}

ns_status ns_spectra_async(ns_ctx* ctx, const void* u_hat, const void* n_hat) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  if (!aligned(u_hat) || (n_hat != nullptr && !aligned(n_hat)))
    return fail(ctx, NS_ERR_ARG, "u_hat (and n_hat if given) must be 256-byte aligned device pointers");
  return ctx->cfg.precision == NS_FP32 ? spectra_enqueue_t<float>(ctx, u_hat, n_hat)
                                       : spectra_enqueue_t<double>(ctx, u_hat, n_hat);
}

ns_status ns_spectra_wait(ns_ctx* ctx, ns_spectra_out* out) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  if (!out) return fail(ctx, NS_ERR_ARG, "out is NULL");
  return spectra_wait(ctx, out);
}

}  // extern "C"

// ---------------------------------------------------------------- spectra without allocation
// ns_spectra_static keeps the FP64 partials and the summed bins in this array: one
// copy per GPU, held until the process ends, shared by every call on that GPU.
// Every entry a call reads is written by the same call first (each block writes all
// of its bins, the second pass every output bin), so nothing needs clearing.
namespace {

constexpr int kStaticMaxN = NS_SPECTRA_STATIC_MAX_N;
constexpr int static_nbins(int n) {
  // 3 shell spectra, 3 one-dimensional spectra of n/2 + 1 bins, 5 totals; shells as num_shells
  return 3 * (int)(1.7320508075688772 * (n / 2) + 2) + 3 * (n / 2 + 1) + 5;
}
constexpr size_t kStaticDoubles = (size_t)(kSpecBlocks + 1) * static_nbins(kStaticMaxN);
__device__ __align__(256) double scratch[kStaticDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up once per device, with the
// device current).
ns_status scratch_for_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, NS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, NS_ERR_STATE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(nullptr, NS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return NS_OK;
}

template <typename R>
ns_status spectra_static_t(int n, double nu, const void* u, const void* nh, hipStream_t stream,
                           ns_spectra_out* out) {
  const int h = n / 2 + 1, nsh = num_shells(n), nbins = 3 * nsh + 3 * h + 5;
  double* base = nullptr;
  ns_status st = scratch_for_current_device(&base);
  if (st != NS_OK) return st;
  double* partials = base;
  double* bins = base + (size_t)kSpecBlocks * nbins;
  const size_t set = (size_t)nbins * sizeof(double);
  const int nwb = (int)std::max<size_t>(1, std::min<size_t>(16, (size_t)(128 * 1024) / set));
  const size_t lds = nwb * set;
  hipError_t e = allow_lds(ns::k_spectra<R>, lds);
  if (e != hipSuccess) return hip_check(nullptr, e, "k_spectra attribute");
  hipLaunchKernelGGL(ns::k_spectra<R>, dim3(kSpecBlocks), dim3(64 * nwb), lds, stream, static_cast<const Cx<R>*>(u),
                     static_cast<const Cx<R>*>(nh), nu, n, h, nsh, (long long)n * n * h, partials);
  hipLaunchKernelGGL(ns::k_spectra_sum, dim3((nbins + 7) / 8), dim3(256), 0, stream, partials, kSpecBlocks, nbins,
                     bins);
  if ((st = hip_check(nullptr, hipGetLastError(), "spectra launch")) != NS_OK) return st;
  double host[static_nbins(kStaticMaxN)];  // on the stack: no host allocation either
  if ((st = hip_check(nullptr, hipMemcpyAsync(host, bins, set, hipMemcpyDeviceToHost, stream), "spectra copy")) !=
      NS_OK)
    return st;
  if ((st = hip_check(nullptr, hipStreamSynchronize(stream), "spectra wait")) != NS_OK) return st;
  if (out->e_shell) std::memcpy(out->e_shell, host, nsh * sizeof(double));
  if (out->d_shell) std::memcpy(out->d_shell, host + nsh, nsh * sizeof(double));
  if (out->t_shell) std::memcpy(out->t_shell, host + 2 * nsh, nsh * sizeof(double));
  if (out->e_1d) std::memcpy(out->e_1d, host + 3 * nsh, 3 * h * sizeof(double));
  if (out->totals) std::memcpy(out->totals, host + 3 * nsh + 3 * h, 5 * sizeof(double));
  if (host[3 * nsh + 3 * h + 4] != 0.0) return fail(nullptr, NS_ERR_NONFINITE, "non-finite entries in input");
  return NS_OK;
}

}  // namespace

extern "C" {

ns_status ns_spectra_static(int32_t n, int32_t precision, double nu, const void* u_hat, const void* n_hat,
                            void* stream, ns_spectra_out* out) {
  if (!factor_ok(n, nullptr)) return fail(nullptr, NS_ERR_ARG, "n must be 2^a 3^b 5^c with a >= 1 and 8 <= n <= 1024");
  if (n > kStaticMaxN)
    return fail(nullptr, NS_ERR_SIZE, "ns_spectra_static supports n <= " + std::to_string(kStaticMaxN) +
                                          " (the size of its static scratch); use ns_spectra");
  if (precision != NS_FP32 && precision != NS_FP64) return fail(nullptr, NS_ERR_ARG, "precision must be NS_FP32 or NS_FP64");
  if (!(nu >= 0.0) || !std::isfinite(nu)) return fail(nullptr, NS_ERR_ARG, "nu must be finite and >= 0");
  if (!aligned(u_hat) || (n_hat != nullptr && !aligned(n_hat)))
    return fail(nullptr, NS_ERR_ARG, "u_hat (and n_hat if given) must be 256-byte aligned device pointers");
  if (!out) return fail(nullptr, NS_ERR_ARG, "out is NULL");
  if (3 * num_shells(n) + 3 * (n / 2 + 1) + 5 > static_nbins(kStaticMaxN))
    return fail(nullptr, NS_ERR_SIZE, "spectra bins exceed the static scratch");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return precision == NS_FP32 ? spectra_static_t<float>(n, nu, u_hat, n_hat, s, out)
                              : spectra_static_t<double>(n, nu, u_hat, n_hat, s, out);
}

ns_status ns_spectra(ns_ctx* ctx, const void* u_hat, const void* n_hat, ns_spectra_out* out) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  if (!out) return fail(ctx, NS_ERR_ARG, "out is NULL");
  ns_status st = ns_spectra_async(ctx, u_hat, n_hat);
  return st != NS_OK ? st : spectra_wait(ctx, out);
}

ns_status ns_timing_enable(ns_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  ctx->timing = enable != 0;
  return NS_OK;
}

ns_status ns_timing_read(ns_ctx* ctx, double* ms, int64_t* launches) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  double acc[NS_NUM_PASSES] = {0};
  int64_t cnt[NS_NUM_PASSES] = {0};
  ns_status st = hip_check(ctx, hipStreamSynchronize(ctx->stream), "timing synchronize");
  if (st != NS_OK) return st;
  for (size_t i = 0; i < ctx->tused; ++i) {
    if (ctx->tpass[i] < 0 || ctx->tpass[i] >= NS_NUM_PASSES) return fail(ctx, NS_ERR_ARG, "pass id out of range");
    float t = 0.f;
    st = hip_check(ctx, hipEventElapsedTime(&t, ctx->events[2 * i], ctx->events[2 * i + 1]), "timing elapsed");
    if (st != NS_OK) return st;
    acc[ctx->tpass[i]] += t;
    cnt[ctx->tpass[i]] += 1;
  }
  ctx->tused = 0;
  for (int k = 0; k < NS_NUM_PASSES; ++k) {
    if (ms) ms[k] = acc[k];
    if (launches) launches[k] = cnt[k];
  }
  return NS_OK;
}

ns_status ns_vjp_rk2_phaseshift(ns_ctx* ctx, const void* u_hat0, void* lam, double dt, int32_t variant,
                                const double alpha[3], const ns_forcing* forcing, int64_t step,
                                const void* stage1) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  if (!aligned(u_hat0) || !aligned(lam)) return fail(ctx, NS_ERR_ARG, "u_hat0 and lam must be non-NULL 256-byte aligned device pointers");
  if (u_hat0 == lam) return fail(ctx, NS_ERR_ARG, "u_hat0 and lam must not overlap");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, NS_ERR_ARG, "dt must be finite and > 0");
  if (variant != NS_PS_EXACT && variant != NS_PS_APPROX && variant != NS_PS_RANDOM)
    return fail(ctx, NS_ERR_ARG, "the adjoint supports NS_PS_EXACT, NS_PS_APPROX and NS_PS_RANDOM only");
  if (variant == NS_PS_RANDOM && (alpha == nullptr || !std::isfinite(alpha[0]) || !std::isfinite(alpha[1]) ||
                                  !std::isfinite(alpha[2])))
    return fail(ctx, NS_ERR_ARG, "NS_PS_RANDOM needs the finite first-stage shift alpha");
  if (ctx->lay.pa == 0) return fail(ctx, NS_ERR_ARG, "the adjoint supports n <= 910");
  if (forcing && variant == NS_PS_EXACT) return fail(ctx, NS_ERR_ARG, "forcing is supported by the Heun variants only");
  ns_status st = check_forcing(ctx, forcing);
  if (st != NS_OK) return st;
  if (stage1 != nullptr) {
    if (variant == NS_PS_EXACT) return fail(ctx, NS_ERR_ARG, "stage1 is kept by the Heun variants only");
    if (!aligned(stage1) || stage1 == lam) return fail(ctx, NS_ERR_ARG, "stage1 must be a 256-byte aligned device array distinct from lam");
  }
  return ctx->cfg.precision == NS_FP32 ? vjp_t<float>(ctx, u_hat0, lam, dt, variant, alpha, forcing, step, stage1)
                                       : vjp_t<double>(ctx, u_hat0, lam, dt, variant, alpha, forcing, step, stage1);
}

ns_status ns_budget_start(ns_ctx* ctx, const void* u_hat) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  if (!aligned(u_hat)) return fail(ctx, NS_ERR_ARG, "u_hat must be a non-NULL 256-byte aligned device pointer");
  ctx->budget = true;
  const ns::Lay U = user_lay(ctx->lay);
  return ctx->cfg.precision == NS_FP32
             ? budget_sample<float>(ctx, static_cast<const Cx<float>*>(u_hat), U, 0.0, false)
             : budget_sample<double>(ctx, static_cast<const Cx<double>*>(u_hat), U, 0.0, false);
}

ns_status ns_budget_stop(ns_ctx* ctx) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  ctx->budget = false;
  return NS_OK;
}

ns_status ns_budget_read(ns_ctx* ctx, double* out) {
  if (!ctx) return fail(nullptr, NS_ERR_ARG, "ctx is NULL");
  if (!out) return fail(ctx, NS_ERR_ARG, "out is NULL");
  ns::Budget b;
  ns_status st = hip_check(ctx, hipMemcpyAsync(&b, ctx->ws + ctx->lay.off_budget, sizeof(b), hipMemcpyDeviceToHost,
                                               ctx->stream), "budget copy");
  if (st == NS_OK) st = hip_check(ctx, hipStreamSynchronize(ctx->stream), "budget wait");
  if (st != NS_OK) return st;
  const double v[NS_BUDGET_LEN] = {b.t, b.E, b.eps, b.E0, b.int_eps, b.int_p, b.p_last, b.residual};
  std::memcpy(out, v, sizeof(v));
  return NS_OK;
}

}  // extern "C"
