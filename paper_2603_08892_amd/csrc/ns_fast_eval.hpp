// ns_fast_eval.hpp -- launch sequences of the specialised FP32 passes of one
// grid size; included by that size's translation unit (fast_<N>.hip), which
// instantiates them for every epilogue and adjoint op with NS_FAST_INSTANTIATE.
#pragma once

#include "ns_host_impl.hpp"

namespace nsh {

template <int N> struct FastOf;
template <> struct FastOf<64> { using type = ns::Fast64; };
template <> struct FastOf<128> { using type = ns::Fast128; };
template <> struct FastOf<192> { using type = ns::Fast192; };
template <> struct FastOf<216> { using type = ns::Fast216; };
template <> struct FastOf<256> { using type = ns::Fast256; };
template <> struct FastOf<324> { using type = ns::Fast324; };
template <> struct FastOf<384> { using type = ns::Fast384; };
template <> struct FastOf<512> { using type = ns::Fast512; };
template <> struct FastOf<144> { using type = ns::Fast144; };
template <> struct FastOf<160> { using type = ns::Fast160; };
template <> struct FastOf<240> { using type = ns::Fast240; };
template <> struct FastOf<270> { using type = ns::Fast270; };
template <> struct FastOf<360> { using type = ns::Fast360; };

// Specialised FP32 passes for one compile-time size (same semantics and layout).
template <typename C, int OP, int FEED>
ns_status eval_fast(ns_ctx* c, const Cx<float>* in, ns::Lay lin, const ns::Shift& sh, const EpiArgs<float>& a,
                    bool front, const ns::Shift& sh2) {
  const Layout& l = c->lay;
  const Geom& g = l.g;
  Ptrs<float> p = ptrs<float>(c);
  constexpr int N = C::N, P = C::PZ;
  hipError_t e;
  const int ntiles = l.ntiles_active;
  if (ntiles > 0) {
    if (front) {
      if ((e = tstart(c, 0)) != hipSuccess) return hip_check(c, e, "timing event");
      hipLaunchKernelGGL((ns::f_xinv<typename C::XInv, !C::YC>), dim3(ntiles), dim3(ns::kFastL * C::XInv::TPL), 0,
                         c->stream, in, lin, p.W, p.tw, sh, p.tiles, g);
      if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
    }
    if ((e = tstart(c, 1)) != hipSuccess) return hip_check(c, e, "timing event");
    if constexpr (C::YC)
      hipLaunchKernelGGL(ns::f_ycurl<typename C::Y>, dim3(2 * N * l.ntz), dim3(ns::kFastL * C::Y::TPL), 0,
                         c->stream, p.W, p.tw, l.ntz, g);
    else
      hipLaunchKernelGGL((ns::f_ypass<typename C::Y, +1>), dim3(6 * N * l.ntz), dim3(ns::kFastL * C::Y::TPL), 0,
                         c->stream, p.W, p.tw, l.ntz, g);
    if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
    if ((e = tstart(c, 2)) != hipSuccess) return hip_check(c, e, "timing event");
    hipLaunchKernelGGL((ns::f_zcross<typename C::Z, P>), dim3(N * N / P), dim3(P * C::Z::TPL), 0, c->stream,
                       p.W, p.tw, g);
    if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
    if ((e = tstart(c, 3)) != hipSuccess) return hip_check(c, e, "timing event");
    hipLaunchKernelGGL((ns::f_ypass<typename C::Y, -1>), dim3(3 * N * l.ntz), dim3(ns::kFastL * C::Y::TPL), 0,
                       c->stream, p.W, p.tw, l.ntz, g);
    if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
  }
  const int nblk = a.full ? N * l.ntzf : ntiles;
  if ((e = tstart(c, FEED ? 5 : 4)) != hipSuccess) return hip_check(c, e, "timing event");
  if (nblk > 0)
    hipLaunchKernelGGL((ns::f_xfwd<typename C::XFwd, OP, FEED, !C::YC>), dim3(nblk),
                       dim3(ns::kFastL * C::XFwd::TPL), 0, c->stream, p.W, p.tw, sh, sh2, p.tiles, g, a);
  if ((e = tstop(c)) != hipSuccess) return hip_check(c, e, "timing event");
  return hip_check(c, hipGetLastError(), "nonlinear-term launch");
}

template <typename C, int OP>
ns_status eval_fast_chain(ns_ctx* c, const Cx<float>* in, ns::Lay lin, const ns::Shift& sh,
                          const EpiArgs<float>& a, Chain* ch) {
  const bool front = !(ch && ch->front_done);
  const int feed = (ch && !a.full && c->lay.ntiles_active > 0) ? ch->feed : 0;
  if (ch) ch->fused = false;
  if constexpr (ns::op_can_feed(OP, 1)) {
    if (feed == 1) {
      ch->fused = true;
      return eval_fast<C, OP, 1>(c, in, lin, sh, a, front, make_shift(ch->next_s));
    }
  }
  if constexpr (ns::op_can_feed(OP, 2)) {
    if (feed == 2) {
      ch->fused = true;
      return eval_fast<C, OP, 2>(c, in, lin, sh, a, front, make_shift(ch->next_s));
    }
  }
  return eval_fast<C, OP, 0>(c, in, lin, sh, a, front, sh);
}

// Specialised FP32 passes of one transposed evaluation (same semantics and layout).
template <typename C, int AOP>
ns_status adj_eval_fast(ns_ctx* c, const Cx<float>* st, ns::Lay lst, const ns::Shift& sh,
                        const LamArgs<float>& la, AdjArgs<float> aa) {
  const Layout& l = c->lay;
  const Geom& g = l.g;
  Ptrs<float> p = ptrs<float>(c);
  constexpr int N = C::N, P = C::PZA;
  const int ntiles = l.ntiles_active;
  if (ntiles > 0) {
    hipLaunchKernelGGL((ns::f_xinv<typename C::XInv, true>), dim3(ntiles), dim3(ns::kFastL * C::XInv::TPL), 0,
                       c->stream, st, lst, p.W, p.tw, sh, p.tiles, g);
    hipLaunchKernelGGL(ns::f_xlam<typename C::XInv>, dim3(ntiles), dim3(ns::kFastL * C::XInv::TPL), 0,
                       c->stream, la, p.W, p.tw, sh, p.tiles, g);
    hipLaunchKernelGGL((ns::f_ypass<typename C::Y, +1>), dim3(9 * N * l.ntz), dim3(ns::kFastL * C::Y::TPL), 0,
                       c->stream, p.W, p.tw, l.ntz, g);
    hipLaunchKernelGGL((ns::f_zadj<typename C::ZAdj, P>), dim3(N * N / P), dim3(P * C::ZAdj::TPL), 0, c->stream,
                       p.W, p.tw, g);
    hipLaunchKernelGGL((ns::f_ypass<typename C::Y, -1>), dim3(6 * N * l.ntz), dim3(ns::kFastL * C::Y::TPL), 0,
                       c->stream, p.W, p.tw, l.ntz, g);
  }
  aa.ntzf = l.ntzf;
  const int nblk = aa.full ? N * l.ntzf : ntiles;
  if (nblk > 0)
    hipLaunchKernelGGL((ns::f_xadj<typename C::XFwd, AOP>), dim3(nblk), dim3(ns::kFastL * C::XFwd::TPL), 0,
                       c->stream, p.W, p.tw, sh, p.tiles, g, aa);
  return hip_check(c, hipGetLastError(), "adjoint launch");
}

template <int N, int OP>
ns_status fast_eval(ns_ctx* c, const Cx<float>* in, ns::Lay lin, const ns::Shift& sh, const EpiArgs<float>& a,
                    Chain* ch) {
  return eval_fast_chain<typename FastOf<N>::type, OP>(c, in, lin, sh, a, ch);
}

template <int N, int AOP>
ns_status fast_adj_eval(ns_ctx* c, const Cx<float>* st, ns::Lay lst, const ns::Shift& sh,
                        const LamArgs<float>& la, AdjArgs<float> aa) {
  return adj_eval_fast<typename FastOf<N>::type, AOP>(c, st, lst, sh, la, aa);
}

}  // namespace nsh

#define NS_FAST_OP(N, OP)                                                                              \
  template ns_status nsh::fast_eval<N, ns::OP>(ns_ctx*, const ns::Cx<float>*, ns::Lay, const ns::Shift&, \
                                               const ns::EpiArgs<float>&, nsh::Chain*);
#define NS_FAST_AOP(N, AOP)                                                                                \
  template ns_status nsh::fast_adj_eval<N, ns::AOP>(ns_ctx*, const ns::Cx<float>*, ns::Lay, const ns::Shift&, \
                                                    const ns::LamArgs<float>&, ns::AdjArgs<float>);
#define NS_FAST_INSTANTIATE(N) \
  NS_FAST_OP(N, OP_STORE) \
  NS_FAST_OP(N, OP_AVG) \
  NS_FAST_OP(N, OP_HEUN1) \
  NS_FAST_OP(N, OP_HEUN2) \
  NS_FAST_OP(N, OP_EX1B) \
  NS_FAST_OP(N, OP_EX2B) \
  NS_FAST_OP(N, OP_RK4_0) \
  NS_FAST_OP(N, OP_RK4_1) \
  NS_FAST_OP(N, OP_RK4_2) \
  NS_FAST_OP(N, OP_RK4_3) \
  NS_FAST_OP(N, OP_ACC) \
  NS_FAST_OP(N, OP_MID1) \
  NS_FAST_OP(N, OP_MID2) \
  NS_FAST_OP(N, OP_EUL) \
  NS_FAST_OP(N, OP_EULAV) \
  NS_FAST_AOP(N, AOP_STORE) \
  NS_FAST_AOP(N, AOP_ACC) \
  NS_FAST_AOP(N, AOP_HEUN) \
  NS_FAST_AOP(N, AOP_EXACT)
