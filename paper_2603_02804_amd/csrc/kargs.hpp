// kargs.hpp -- argument records of the device kernels and the host code that
// fills them from a plan.  Plain structs of pointers and integers, shared by the
// single-plan launch backend, the merged mixed-batch programs and the CPU checker.
#pragma once
#include <stdint.h>

#include <algorithm>

#include "driver.hpp"

namespace qf {

// Device addresses of a plan's read-only tables.
struct Tabs {
  const EventRec* events;
  const RunRec* runs;
  const int32_t* run_gates;
  const GateRec* gates;
  const int32_t* coef_runs_sh;
  const int32_t* coef_runs_ps;
  const PassRec* passes;
  const int64_t* partF_off;
  const int32_t* seg_runs;
  const int32_t* seg_run_begin;
  const int32_t* th_ref_begin;
  const int32_t* th_refs;
  const int32_t* in_ref_begin;
  const int32_t* in_refs;
  const int32_t* pass_run_begin;
  const int32_t* pass_runs;
};

struct PlanPtrs {
  const Op* ops = nullptr;
  const LayoutRec* layouts = nullptr;
  const CzGroup* czg = nullptr;
  const FuncEntry* funcs = nullptr;
  const RygEntry* rygs = nullptr;
  const EpochRec* epochs = nullptr;
  const PhaEntry* phas = nullptr;
  const PassRec* passes = nullptr;
  const uint32_t* zmask = nullptr;
  const PhaseEv* pev = nullptr;
  const CzaRec* cza = nullptr;
  Tabs tabs{};
};

// Fused pass: one workgroup per (sample, tile).
struct KArgs {
  const Op* ops;
  const LayoutRec* layouts;
  const CzGroup* czg;
  const FuncEntry* funcs;
  const RygEntry* rygs;
  const EpochRec* epochs;
  const PhaEntry* phas;
  const PassRec* prec;
  const PhaseEv* pev;
  const CzaRec* cza;
  const float* coef_sh;
  const float* coef_ps;
  const float* ev_sh;
  const float* ev_ps;
  const float* src0;          // psi input, interleaved complex
  const float* src1;          // lambda input
  float* dst;
  float* partF;
  float* partE;
  const float* dE;
  const uint32_t* zmask;
  long long s0, s1, sd;       // per-sample strides (complex elements)
  int n_ops;
  int n_ps;                   // per-sample run coefficient rows per sample
  int n_evps;                 // per-sample phase event rows per sample
  int K;
  int sample0;
  int tiles_log2;
  int tb;                     // thread bits of the tile
  int do_expect;
  int tile_elems;             // 2^k: LDS elements of the tile; wave partial sums follow
};

struct CoefArgs {
  Tabs T;
  const float* theta;
  const float* x;
  float* csh;
  float* cps;
  int F, n_sh, n_ps, B, zyz;
};

struct EventArgs {
  Tabs T;
  const float* csh;
  const float* cps;
  float* esh;
  float* eps;
  int n_ev_sh, n_ev_ps, B, n_ps;
};

struct ReduceEArgs {
  const float* partE;
  float* E;
  int nb, sample0, parts, K;
};

struct AssembleArgs {
  Tabs T;
  const float* theta;
  const float* x;
  const float* partF;
  float* Gr;
  int p0, np, nb, sample0, tiles, n_angle, F;
};

struct ReduceGArgs {
  Tabs T;
  const float* Gr;
  float* dtheta;
  float* dx;
  int nb, sample0, n_angle, P, F, accumulate;
};

constexpr int kSmallThreads = 256;

inline unsigned blocks_for(long long n, int t = kSmallThreads) {
  return (unsigned)std::max<long long>(1, (n + t - 1) / t);
}

// Workspace addresses of the coefficient tables of one call.
struct CoefPtrs {
  const float* csh = nullptr;
  const float* cps = nullptr;
  const float* esh = nullptr;
  const float* eps = nullptr;
};

inline CoefPtrs coef_ptrs(const PlanCore& c, char* ws) {
  CoefPtrs p;
  p.csh = at<float>(ws, c.off_coef_sh);
  p.cps = at<float>(ws, c.off_coef_ps);
  p.esh = at<float>(ws, c.off_ev_sh);
  p.eps = at<float>(ws, c.off_ev_ps);
  return p;
}

inline KArgs make_pass_args(const PlanCore& c, const PlanPtrs& d, const CoefPtrs& cp, const PassLaunch& L) {
  const Schedule& S = c.S;
  const PassRec& pr = S.passes[L.pass];
  KArgs A;
  A.ops = d.ops + (L.bwd ? pr.bop_begin : pr.fop_begin);
  A.n_ops = L.bwd ? pr.bop_count : pr.fop_count;
  A.layouts = d.layouts;
  A.czg = d.czg;
  A.funcs = d.funcs;
  A.rygs = d.rygs;
  A.epochs = d.epochs;
  A.phas = d.phas;
  A.prec = d.passes + L.pass;
  A.pev = d.pev;
  A.cza = d.cza;
  A.coef_sh = cp.csh;
  A.coef_ps = cp.cps;
  A.ev_sh = cp.esh;
  A.ev_ps = cp.eps;
  A.n_ps = S.n_coef_ps;
  A.n_evps = S.n_ev_ps;
  A.src0 = L.src0;
  A.s0 = L.src0_stride / 2;
  A.src1 = L.src1;
  A.s1 = L.src1_stride / 2;
  A.dst = L.dst;
  A.sd = L.dst_stride / 2;
  A.partF = L.partF;
  A.partE = L.partE;
  A.dE = L.dE;
  A.zmask = d.zmask;
  A.K = c.C.K;
  A.sample0 = L.sample0;
  A.tiles_log2 = S.tiles_log2;
  A.tb = S.thread_bits;
  A.do_expect = L.do_expect;
  A.tile_elems = 1 << S.k;
  return A;
}

inline unsigned pass_blocks(const PlanCore& c, int nb) { return (unsigned)((long long)nb << c.S.tiles_log2); }

// Dynamic LDS of a pass workgroup (the tile itself is a static array of the
// kernel): backward only, one partial sum per wave, functional slot and Pauli.
inline size_t pass_shmem(const PlanCore& c, bool bwd) {
  const Schedule& S = c.S;
  return bwd ? sizeof(float) * 3 * S.max_slots * (S.NT / 64) : 0;
}

inline CoefArgs make_coef_args(const PlanCore& c, const PlanPtrs& d, const float* theta, const float* x,
                               const CoefPtrs& cp) {
  CoefArgs a;
  a.T = d.tabs;
  a.theta = theta;
  a.x = x;
  a.csh = const_cast<float*>(cp.csh);
  a.cps = const_cast<float*>(cp.cps);
  a.F = c.C.F;
  a.n_sh = c.S.n_coef_shared;
  a.n_ps = c.S.n_coef_ps;
  a.B = c.B;
  a.zyz = c.per_gate ? 0 : 1;
  return a;
}

inline long long coef_items(const CoefArgs& a) { return a.n_sh + (long long)a.n_ps * a.B; }

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

inline ReduceEArgs make_reduce_E_args(const PlanCore& c, int nb, int sample0, int parts, const float* partE,
                                      float* E) {
  ReduceEArgs a;
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

inline ReduceGArgs make_reduce_grads_args(const PlanCore& c, const PlanPtrs& d, int nb, int sample0,
                                          const float* Gr, float* dtheta, float* dx, bool accumulate) {
  ReduceGArgs a;
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
  return a;
}

inline long long reduce_grads_items(const ReduceGArgs& a) { return a.P + (long long)a.nb * a.F; }

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
