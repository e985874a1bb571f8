// kargs.hpp -- argument record of the fused pass kernels and the host code that
// fills it from a plan.  Plain structs of pointers and integers, shared by the
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
  const double* consts;         // fixed angles of internal gates (lowered CNOT)
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
  const PauliRec* pauli = nullptr;   // observables in the final state's bit order
  const ThrBase* tbases = nullptr;   // [layout][thread] bases (S.NT threads per layout)
  Tabs tabs{};
};

// Fused pass: one workgroup per (sample, tile).
struct KArgs {
  const Op* ops;
  const LayoutRec* layouts;
  const ThrBase* tbases;      // [layout][NT] thread bases of every layout
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
  uint32_t* dst2;             // forward: bfloat16-pair copy of the output (memory-saving mode)
  long long sd2;              // its per-sample stride (words)
  int src0_bf16;              // psi input as bfloat16 pairs (4 bytes per amplitude)
  float* dpsi;                // backward: psi at the pass input (uncompute mode), or null
  long long sdp;              // its per-sample stride (complex elements)
};

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
  A.ops = d.ops + (L.bwd ? pr.bop_begin : (L.load_input ? pr.fload_begin : pr.fop_begin));
  A.n_ops = L.bwd ? pr.bop_count : pr.fop_count;
  A.layouts = d.layouts;
  A.tbases = d.tbases;
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
  A.s0 = L.src0_bf16 ? L.src0_stride : L.src0_stride / 2;
  A.src0_bf16 = L.src0_bf16 ? 1 : 0;
  A.src1 = L.src1;
  A.s1 = L.src1_stride / 2;
  A.dst = L.dst;
  A.sd = L.dst_stride / 2;
  A.dst2 = L.dst2;
  A.sd2 = L.dst2_stride;
  A.dpsi = L.dpsi;
  A.sdp = L.dpsi_stride / 2;
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

}  // namespace qf
