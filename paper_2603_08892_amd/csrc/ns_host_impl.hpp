// ns_host_impl.hpp -- host-side internals shared by the translation units of
// libns.so: the workspace layout, the context, error and timing helpers, and the
// entry points of the specialised FP32 passes (one translation unit per size,
// ns_fast_eval.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <new>
#include <string>
#include <vector>

#include "../../include/ns.h"
#include "ns_adjoint.hpp"
#include "ns_fast.hpp"
#include "ns_fast_adjoint.hpp"
#include "ns_aux_types.hpp"

namespace nsh {

using ns::Cx;
using ns::EpiArgs;
using ns::FftPlan;
using ns::Geom;
using ns::AdjArgs;
using ns::LamArgs;

constexpr int kEpt = 8;     // points per thread in the strided passes
constexpr int kEptZ = 16;   // points per thread in the contiguous (z) pass
constexpr size_t kAlign = 256;
constexpr int kSpecBlocks = 256;  // one block per CU; its wavefronts keep private LDS bins

// message of the last failure of a call without a context, per thread
extern thread_local std::string g_last_error;

struct Layout {
  Geom g;
  FftPlan plan;
  int elem;          // bytes per complex element
  int tx;            // threads of the strided passes
  int ntz;           // k_z tiles over [0, kzn)
  int ntzf;          // k_z tiles over [0, N/2]
  int pz, tz;        // lines per block and threads of the z pass
  int pa, ta;        // the same for the adjoint z pass (0: adjoint not available)
  long long k2top;   // largest retained |k|^2
  int nsh, nbins;
  std::vector<int2> tiles;   // active (k_y index, k_z tile start)
  int ntiles_active;
  size_t off_tw, off_etab, off_force, off_tiles, off_w, off_s, off_a, off_spec, off_specout;
  size_t off_fstate, off_budget, off_bpart;  // forcing record, budget record, budget partials
  size_t total;
};

}  // namespace nsh

struct ns_ctx {
  ns_config cfg;
  hipStream_t stream;
  nsh::Layout lay;
  char* ws;
  std::string err;
  double* pin_spec = nullptr;    // pinned host copy of the last spectra reduction
  hipEvent_t spec_ev = nullptr;  // recorded after that copy
  bool spec_pending = false;     // a reduction was enqueued and not yet waited for
  int fast = 0;       // N of the specialised FP32 passes in use (0: generic passes)
  double etab_dt = -1.0;  // dt of the integrating-factor tables now in the workspace
  // per-pass timing: events[2 i], events[2 i + 1] bracket launch i of pass tpass[i]
  bool budget = false;     // update the energy budget after every step
  bool timing = false;
  std::vector<hipEvent_t> events;
  std::vector<int> tpass;
  size_t tused = 0;
  ~ns_ctx() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (spec_ev) (void)hipEventDestroy(spec_ev);
    if (pin_spec) (void)hipHostFree(pin_spec);
  }
};

namespace nsh {

inline ns_status fail(ns_ctx* c, ns_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_last_error = msg;
  return s;
}

inline ns_status hip_check(ns_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return NS_OK;
  return fail(c, NS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

inline bool aligned(const void* p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

// Timing brackets around one pass launch (no-ops unless timing is enabled).
inline hipError_t tstart(ns_ctx* c, int pass) {
  if (!c->timing) return hipSuccess;
  if (pass < 0 || pass >= NS_NUM_PASSES) return hipErrorInvalidValue;  // ns_timing_read indexes by pass
  if (2 * c->tused + 2 > c->events.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      c->events.push_back(e);
    }
    c->tpass.push_back(pass);
  }
  c->tpass[c->tused] = pass;
  return hipEventRecord(c->events[2 * c->tused], c->stream);
}

inline hipError_t tstop(ns_ctx* c) {
  if (!c->timing) return hipSuccess;
  hipError_t r = hipEventRecord(c->events[2 * c->tused + 1], c->stream);
  ++c->tused;
  return r;
}

template <typename R>
struct Ptrs {
  Cx<R>* tw;
  R* eh;
  R* edt;
  Cx<R>* force;
  int2* tiles;
  Cx<R>* W;
  Cx<R>* sb;
  Cx<R>* ab;
  double* spec;
  double* specout;
  ns::ForceState* fstate;
  ns::Budget* budget;
  double* bpart;
};

template <typename R>
Ptrs<R> ptrs(ns_ctx* c) {
  const Layout& l = c->lay;
  Ptrs<R> p;
  p.tw = reinterpret_cast<Cx<R>*>(c->ws + l.off_tw);
  p.eh = reinterpret_cast<R*>(c->ws + l.off_etab);
  p.edt = p.eh + (l.k2top + 1);
  p.force = reinterpret_cast<Cx<R>*>(c->ws + l.off_force);
  p.tiles = reinterpret_cast<int2*>(c->ws + l.off_tiles);
  p.W = reinterpret_cast<Cx<R>*>(c->ws + l.off_w);
  p.sb = reinterpret_cast<Cx<R>*>(c->ws + l.off_s);
  p.ab = reinterpret_cast<Cx<R>*>(c->ws + l.off_a);
  p.spec = reinterpret_cast<double*>(c->ws + l.off_spec);
  p.specout = reinterpret_cast<double*>(c->ws + l.off_specout);
  p.fstate = reinterpret_cast<ns::ForceState*>(c->ws + l.off_fstate);
  p.budget = reinterpret_cast<ns::Budget*>(c->ws + l.off_budget);
  p.bpart = reinterpret_cast<double*>(c->ws + l.off_bpart);
  return p;
}

inline size_t lds_strided(const Layout& l) { return (size_t)(2 * l.g.n + l.g.n * l.g.L) * l.elem; }

// Layouts: the caller's arrays and the compact internal stage buffers.
inline ns::Lay user_lay(const Layout& l) { return ns::Lay{l.g.h, l.g.comp}; }
inline ns::Lay compact_lay(const Layout& l) { return ns::Lay{l.g.kzp, l.g.wcomp}; }
inline ns::Shift make_shift(const double* s) {
  ns::Shift sh;
  sh.s[0] = s ? s[0] : 0.0;
  sh.s[1] = s ? s[1] : 0.0;
  sh.s[2] = s ? s[2] : 0.0;
  sh.on = (s != nullptr && (s[0] != 0.0 || s[1] != 0.0 || s[2] != 0.0)) ? 1 : 0;
  return sh;
}
inline size_t lds_z(const Layout& l) { return (size_t)(l.g.n + 3 * l.pz * l.g.n) * l.elem; }
inline size_t lds_zadj(const Layout& l) { return (size_t)(l.g.n + (9 * l.pa * l.g.n) / 2) * l.elem; }

template <typename K>
inline hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename R, int OP>
inline hipError_t launch_xfwd(ns_ctx* c, const Ptrs<R>& p, const ns::Shift& sh, const EpiArgs<R>& a) {
  const Layout& l = c->lay;
  const size_t lds = lds_strided(l);
  auto kern = ns::k_xfwd<R, kEpt, OP>;
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int nblk = a.full ? l.g.n * l.ntzf : l.ntiles_active;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3(nblk), dim3(l.tx), lds, c->stream, p.W, p.tw, sh, p.tiles, l.g, l.plan, a);
  return hipGetLastError();
}

// Chaining of consecutive evaluations.  In: front_done = this evaluation's
// x-inverse pass already ran (fused into the previous x-forward pass); feed = the
// stage output that is the next evaluation's input (0 none, 1 out0, 2 out1) and
// next_s its shift.  Out: fused = the next evaluation's x-inverse pass ran here
// (only the specialised passes fuse, and only into a stage that is not in full
// mode); an out1 that feeds is then not stored.
struct Chain {
  bool front_done = false;
  int feed = 0;
  const double* next_s = nullptr;
  bool fused = false;
};

// Specialised FP32 passes of size N (defined and instantiated for every op in the
// translation unit of that size): one evaluation of the nonlinear term, and one
// transposed evaluation.
template <int N, int OP>
ns_status fast_eval(ns_ctx* c, const Cx<float>* in, ns::Lay lin, const ns::Shift& sh, const EpiArgs<float>& a,
                    Chain* ch);
template <int N, int AOP>
ns_status fast_adj_eval(ns_ctx* c, const Cx<float>* st, ns::Lay lst, const ns::Shift& sh,
                        const LamArgs<float>& la, AdjArgs<float> aa);

}  // namespace nsh
