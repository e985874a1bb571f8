// small_args.hpp -- argument records of the coefficient, assembly and
// reduction kernels, the host code that fills them from a plan, and the job
// records of merged mixed-batch launches.
#pragma once
#include <stdint.h>

#include <algorithm>

#include "kargs.hpp"

namespace qf {

// Coefficient, reduction and gradient arguments carry the real type of the call:
// float on the fused and per-gate paths, double on the complex128 validation path.
template <class Real>
struct CoefArgsT {
  Tabs T;
  const Real* theta;
  const Real* x;
  Real* csh;
  Real* cps;
  int F, n_sh, n_ps, B, zyz;
};
using CoefArgs = CoefArgsT<float>;

struct EventArgs {
  Tabs T;
  const float* csh;
  const float* cps;
  float* esh;
  float* eps;
  int n_ev_sh, n_ev_ps, B, n_ps;
};

template <class Real>
struct ReduceEArgsT {
  const Real* partE;
  Real* E;
  int nb, sample0, parts, K;
};
using ReduceEArgs = ReduceEArgsT<float>;

struct AssembleArgs {
  Tabs T;
  const float* theta;
  const float* x;
  const float* partF;
  float* Gr;
  int p0, np, nb, sample0, tiles, n_angle, F;
};

template <class Real>
struct ReduceGArgsT {
  Tabs T;
  const Real* Gr;
  Real* dtheta;
  Real* dx;
  int nb, sample0, n_angle, P, F, accumulate;
  // dtheta blocks: each sums cols angles over the micro-batch with kSmallThreads / cols
  // sample lanes (lane j takes samples j, j + lanes, ...), then a fixed tree over the lanes
  int cols, th_blocks;
  // (the dx pointer of a mixed batch is only known at call time: items are counted regardless)
  long long dx_items() const { return (long long)nb * F; }
};
using ReduceGArgs = ReduceGArgsT<float>;

constexpr int kSmallThreads = 256;

inline unsigned blocks_for(long long n, int t = kSmallThreads) {
  return (unsigned)std::max<long long>(1, (n + t - 1) / t);
}

template <class Real>
inline CoefArgsT<Real> make_coef_args_t(const PlanCore& c, const PlanPtrs& d, const Real* theta, const Real* x,
                                        Real* csh, Real* cps) {
  CoefArgsT<Real> a;
  a.T = d.tabs;
  a.theta = theta;
  a.x = x;
  a.csh = csh;
  a.cps = cps;
  a.F = c.C.F;
  a.n_sh = c.S.n_coef_shared;
  a.n_ps = c.S.n_coef_ps;
  a.B = c.B;
  a.zyz = c.per_gate ? 0 : 1;
  return a;
}

inline CoefArgs make_coef_args(const PlanCore& c, const PlanPtrs& d, const float* theta, const float* x,
                               const CoefPtrs& cp) {
  return make_coef_args_t<float>(c, d, theta, x, const_cast<float*>(cp.csh), const_cast<float*>(cp.cps));
}

template <class Real>
inline long long coef_items(const CoefArgsT<Real>& a) { return a.n_sh + (long long)a.n_ps * a.B; }

inline EventArgs make_event_args(const PlanCore& c, const PlanPtrs& d, const CoefPtrs& cp) {
  EventArgs a;
  a.T = d.tabs;
  a.csh = cp.csh;
  a.cps = cp.cps;
  a.esh = const_cast<float*>(cp.esh);
  a.eps = const_cast<float*>(cp.eps);
  a.n_ev_sh = c.S.n_ev_shared;
  a.n_ev_ps = c.S.n_ev_ps;
  a.B = c.B;
  a.n_ps = c.S.n_coef_ps;
  return a;
}

inline long long event_items(const EventArgs& a) { return a.n_ev_sh + (long long)a.n_ev_ps * a.B; }

template <class Real>
inline ReduceEArgsT<Real> make_reduce_E_args(const PlanCore& c, int nb, int sample0, int parts, const Real* partE,
                                             Real* E) {
  ReduceEArgsT<Real> a;
  a.partE = partE;
  a.E = E;
  a.nb = nb;
  a.sample0 = sample0;
  a.parts = parts;
  a.K = c.C.K;
  return a;
}

inline AssembleArgs make_assemble_args(const PlanCore& c, const PlanPtrs& d, int seg, int nb, int sample0,
                                       const float* theta, const float* x, const float* partF, float* Gr) {
  AssembleArgs a;
  a.T = d.tabs;
  a.theta = theta;
  a.x = x;
  a.partF = partF;
  a.Gr = Gr;
  a.p0 = c.seg_begin[seg];
  a.np = c.seg_begin[seg + 1] - a.p0;
  a.nb = nb;
  a.sample0 = sample0;
  a.tiles = c.tiles;
  a.n_angle = c.n_angle;
  a.F = c.C.F;
  return a;
}

inline size_t assemble_shmem(const PlanCore& c) { return sizeof(double) * 3 * std::max(1, c.S.max_slots); }

template <class Real>
inline ReduceGArgsT<Real> make_reduce_grads_args(const PlanCore& c, const PlanPtrs& d, int nb, int sample0,
                                                 const Real* Gr, Real* dtheta, Real* dx, bool accumulate) {
  ReduceGArgsT<Real> a;
  a.T = d.tabs;
  a.Gr = Gr;
  a.dtheta = dtheta;
  a.dx = dx;
  a.nb = nb;
  a.sample0 = sample0;
  a.n_angle = c.n_angle;
  a.P = c.C.P;
  a.F = c.C.F;
  a.accumulate = accumulate ? 1 : 0;
  // wide blocks of angles when there are many (coalesced rows of Gr), more sample
  // lanes per angle when there are few
  int cols = 1;
  while (cols < 64 && cols < a.P) cols *= 2;
  a.cols = cols;
  a.th_blocks = (a.P + cols - 1) / cols;
  return a;
}

// Blocks of kSmallThreads threads: th_blocks for dtheta, then one thread per
// (sample, input) for dx.
template <class Real>
inline long long reduce_grads_blocks(const ReduceGArgsT<Real>& a) {
  const long long nx = a.dx_items();
  return (long long)a.th_blocks + (nx + kSmallThreads - 1) / kSmallThreads;
}
inline size_t reduce_grads_shmem() { return sizeof(double) * kSmallThreads; }

// ---------------------------------------------------------------- mixed batches
// Caller buffers of one circuit of a mixed batch, refreshed on every call.
struct CircPtrs {
  const float* theta;
  const float* x;
  float* E;
  const float* dE;
  float* dtheta;
  float* dx;
};

// A pass launch of one circuit inside a merged launch.  Workspace addresses are
// stored as offsets from the batch workspace base (never 0: the first bytes of
// the workspace are reserved), null stays null; dE comes from CircPtrs.
struct PassJob {
  KArgs A;
  int32_t circ;
  int32_t pass;       // pass index in the circuit's plan (host checks only)
};

enum SmallKind : int32_t { SJ_COEF = 0, SJ_EVENT = 1, SJ_REDUCE_E = 2, SJ_ASSEMBLE = 3, SJ_REDUCE_G = 4 };

// A small-kernel launch of one circuit inside a merged launch: same address
// convention; theta, x, E, dtheta and dx come from CircPtrs.
struct SmallJob {
  int32_t kind;
  int32_t circ;
  union {
    CoefArgs coef;
    EventArgs ev;
    ReduceEArgs re;
    AssembleArgs as;
    ReduceGArgs rg;
  } u;
};

}  // namespace qf
