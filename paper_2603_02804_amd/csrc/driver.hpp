// driver.hpp -- sequencing of one forward / backward call over passes,
// checkpoint segments and micro-batches, written once for any backend that
// provides the launch methods used below.
//
// Gradient checkpointing (Sec. 3.4): the forward keeps the state at the end of
// every segment of `ckpt` consecutive fused passes.  The backward walks the
// segments in reverse; for each it re-runs the segment's forward passes from the
// previous checkpoint, storing every pass output (the fused outputs of Sec. 3.2),
// then runs the fused adjoint passes in reverse order (Sec. 3.3).  Within a pass
// the intermediate states are recomputed in registers by un-applying the runs.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "plan.hpp"

namespace qf {

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

struct PassLaunch {
  int pass = 0;
  bool bwd = false;
  int nb = 0;               // samples in this launch
  int sample0 = 0;          // global index of the first sample
  const float* src0 = nullptr; int64_t src0_stride = 0;   // psi input  (interleaved complex)
  const float* src1 = nullptr; int64_t src1_stride = 0;   // lambda input
  float* dst = nullptr; int64_t dst_stride = 0;           // psi (fwd) or lambda (bwd) output
  // memory-saving mode: strides count 4-byte words (2 per complex64 amplitude,
  // 1 per bfloat16 pair)
  bool src0_bf16 = false;   // psi input stored as bfloat16 pairs
  uint32_t* dst2 = nullptr; int64_t dst2_stride = 0;      // forward: bfloat16 copy of the output
  float* dpsi = nullptr; int64_t dpsi_stride = 0;         // backward: psi at the pass input (uncompute)
  float* partF = nullptr;   // backward functional partial sums of this pass: [sample][tile][slot][3]
  float* partE = nullptr;   // forward expectation partial sums
  const float* dE = nullptr;
  int do_expect = 0;
  bool load_input = false;  // pass 0 reads a caller's initial state from src0
};

struct PlanCore {
  Circuit C;
  Tuning T;
  Schedule S;
  int B = 0;
  bool per_gate = false;              // one kernel per gate (float baseline or complex128)
  bool c128 = false;                  // complex128 validation path (double throughout)
  int P = 0, ckpt = 1, n_seg = 1, mb = 1, store = 1;
  int memsave = 0;                    // stored pass outputs of the active segment in bfloat16
  int uncompute = 0;                  // adjoint passes write psi at their input: no recompute
  int waves = 1, tiles = 1;
  int64_t amps = 1;                   // 2^n
  size_t state_bytes = 8;
  int n_angle = 0;
  std::vector<int32_t> seg_begin;     // n_seg + 1 pass indices
  std::vector<int32_t> coef_runs_sh, coef_runs_ps;
  std::vector<int64_t> partF_off;     // per pass, floats, from the start of its segment
  int64_t partF_seg_floats = 0;       // per sample, largest segment
  std::vector<int32_t> seg_runs, seg_run_begin;
  std::vector<int32_t> th_ref_begin, th_refs, in_ref_begin, in_refs;
  // per-gate baseline
  int pg_chunk = 0;                   // rotation gates per partial-sum chunk
  int pg_blocks = 0;                  // partial sums per sample per gate
  int pauli_blocks = 1;               // partial sums per sample of the Pauli-string expectation
  // workspace
  size_t off_coef_sh = 0, off_coef_ps = 0, off_ev_sh = 0, off_ev_ps = 0;
  size_t off_ckpt = 0, off_work = 0, off_seg = 0, off_lam = 0;
  size_t off_partE = 0, off_partF = 0, off_Gr = 0, ws_bytes = 0;
};

// Shape of one per-gate kernel launch: pairs per thread and threads per block.
constexpr int kPgThreads = 256;
constexpr int kPgPairsPerThread = 4;
// Amplitudes per thread of the Pauli-string expectation kernel.
constexpr int kPauliAmpsPerThread = 8;

inline void build_csr(int n_keys, const std::vector<std::pair<int, int>>& kv, std::vector<int32_t>* begin,
                      std::vector<int32_t>* vals) {
  begin->assign(n_keys + 1, 0);
  for (auto& p : kv) (*begin)[p.first + 1]++;
  for (int i = 0; i < n_keys; ++i) (*begin)[i + 1] += (*begin)[i];
  vals->assign(kv.size(), 0);
  std::vector<int32_t> fill(begin->begin(), begin->end() - 1);
  for (auto& p : kv) (*vals)[fill[p.first]++] = p.second;
}

// Builds the schedule and every host-side table and workspace offset.
inline qf_status build_plan_core(const Circuit& C, int B, const Tuning& T, PlanCore* pc, std::string* msg) {
  PlanCore& c = *pc;
  c = PlanCore{};
  c.C = C;
  c.T = T;
  c.B = B;
  c.per_gate = (T.mode == 1 || T.mode == 2);
  c.c128 = (T.mode == 2);
  const size_t real_bytes = c.c128 ? sizeof(double) : sizeof(float);
  c.amps = int64_t(1) << C.n;
  c.state_bytes = (2 * real_bytes) << C.n;
  if (c.per_gate) {
    build_gate_runs(C, &c.S);
    c.S.n = C.n;
  } else if (!build_schedule(C, T, &c.S, msg)) {
    return QF_ERR_INTERNAL;
  }
  const Schedule& S = c.S;
  c.n_angle = (int)S.gates.size();
  for (size_t r = 0; r < S.runs.size(); ++r) {
    if (S.runs[r].coef >= 0) c.coef_runs_sh.push_back((int)r);
    else c.coef_runs_ps.push_back((int)r);
  }
  // gradient references (CSR): theta index -> gate rows, input index -> gate rows
  std::vector<std::pair<int, int>> th, in;
  for (size_t g = 0; g < S.gates.size(); ++g) {
    if (S.gates[g].theta_idx >= 0) th.push_back({S.gates[g].theta_idx, (int)g});
    else if (S.gates[g].input_idx >= 0) in.push_back({S.gates[g].input_idx, (int)g});
  }
  build_csr(C.P, th, &c.th_ref_begin, &c.th_refs);
  build_csr(C.F, in, &c.in_ref_begin, &c.in_refs);

  const size_t SB = c.state_bytes;
  c.pauli_blocks = (int)std::max<int64_t>(1, (c.amps + int64_t(kPgThreads) * kPauliAmpsPerThread - 1) /
                                                  (int64_t(kPgThreads) * kPauliAmpsPerThread));
  if (c.per_gate) {
    c.mb = T.micro > 0 ? std::min(T.micro, B) : std::min(B, 8);
    const int64_t pairs = std::max<int64_t>(1, c.amps / 2);
    const int64_t per_block = int64_t(kPgThreads) * kPgPairsPerThread;
    c.pg_blocks = (int)((pairs + per_block - 1) / per_block);
    c.pg_chunk = std::max(1, std::min(c.n_angle, 4096));
    const size_t rb = real_bytes;
    size_t off = 0;
    c.off_coef_sh = off; off = align_up(off + rb * 8 * std::max(1, S.n_coef_shared));
    c.off_coef_ps = off; off = align_up(off + rb * 8 * std::max<int64_t>(1, int64_t(B) * S.n_coef_ps));
    c.off_ev_sh = off;   off = align_up(off + rb * 2);
    c.off_ev_ps = off;   off = align_up(off + rb * 2);
    c.off_ckpt = off;    off = align_up(off + SB * B);            // final states of the batch
    c.off_lam = off;     off = align_up(off + SB * 2 * c.mb);     // psi copy + lambda
    c.off_partE = off;   off = align_up(off + rb * std::max<int64_t>(1, int64_t(c.mb) * c.pauli_blocks * C.K));
    c.off_partF = off;   off = align_up(off + rb * int64_t(c.mb) * c.pg_chunk * c.pg_blocks * 3);
    c.off_Gr = off;      off = align_up(off + rb * std::max<int64_t>(1, int64_t(c.mb) * c.n_angle));
    c.ws_bytes = off;
    return QF_OK;
  }

  c.P = (int)S.passes.size();
  c.tiles = 1 << S.tiles_log2;
  c.waves = std::max(1, S.NT / 64);
  // checkpoint segments (passes per segment) and micro-batch
  c.ckpt = T.ckpt > 0 ? std::min(T.ckpt, c.P) : std::max(1, (int)std::lround(std::sqrt((double)c.P)));
  c.n_seg = (c.P + c.ckpt - 1) / c.ckpt;
  c.seg_begin.resize(c.n_seg + 1);
  for (int s = 0; s <= c.n_seg; ++s) c.seg_begin[s] = std::min(c.P, s * c.ckpt);
  if (T.micro > 0) {
    c.mb = std::min(T.micro, B);
  } else {
    // enough workgroups to fill the device many times over (short passes are
    // bound by the tail of each launch otherwise), bounded by memory
    const int want_items = 16384;
    int m = std::max(1, want_items / c.tiles);
    const size_t budget = size_t(16) << 30;
    const size_t per_sample = SB * (size_t)(c.ckpt + 4);
    m = (int)std::min<size_t>(m, std::max<size_t>(1, budget / per_sample));
    c.mb = std::max(1, std::min(m, B));
  }
  c.store = T.store >= 0 ? (T.store ? 1 : 0) : 1;
  c.memsave = T.memsave ? 1 : 0;
  c.uncompute = T.uncompute > 0 ? 1 : 0;
  // partial-sum offsets per pass, relative to the segment start
  c.partF_off.assign(c.P, 0);
  for (int s = 0; s < c.n_seg; ++s) {
    int64_t acc = 0;
    for (int p = c.seg_begin[s]; p < c.seg_begin[s + 1]; ++p) {
      c.partF_off[p] = acc;
      acc += int64_t(c.tiles) * 3 * S.passes[p].n_slots;
    }
    c.partF_seg_floats = std::max(c.partF_seg_floats, acc);
  }
  // runs per segment
  c.seg_run_begin.assign(c.n_seg + 1, 0);
  std::vector<std::vector<int32_t>> per_seg(c.n_seg);
  for (size_t r = 0; r < S.runs.size(); ++r) {
    int s = S.runs[r].pass / c.ckpt;
    per_seg[s].push_back((int)r);
  }
  for (int s = 0; s < c.n_seg; ++s) {
    c.seg_run_begin[s] = (int)c.seg_runs.size();
    c.seg_runs.insert(c.seg_runs.end(), per_seg[s].begin(), per_seg[s].end());
  }
  c.seg_run_begin[c.n_seg] = (int)c.seg_runs.size();

  size_t off = 0;
  const int nck = c.store ? B : c.mb;
  c.off_coef_sh = off; off = align_up(off + sizeof(float) * 8 * std::max(1, S.n_coef_shared));
  c.off_coef_ps = off; off = align_up(off + sizeof(float) * 8 * std::max<int64_t>(1, int64_t(B) * S.n_coef_ps));
  c.off_ev_sh = off;   off = align_up(off + sizeof(float) * 2 * std::max(1, S.n_ev_shared));
  c.off_ev_ps = off;   off = align_up(off + sizeof(float) * 2 * std::max<int64_t>(1, int64_t(B) * S.n_ev_ps));
  c.off_ckpt = off;    off = align_up(off + SB * size_t(nck) * c.n_seg);
  c.off_work = off;    off = align_up(off + SB * size_t(c.mb) * 2);
  c.off_seg = off;     off = align_up(off + (c.uncompute ? 0 : (c.memsave ? SB / 2 : SB) * size_t(c.mb) *
                                                               std::max(0, c.ckpt - 1)));
  c.off_lam = off;     off = align_up(off + SB * size_t(c.mb) * 2);
  c.off_partE = off;   off = align_up(off + sizeof(float) * std::max<int64_t>(1, int64_t(c.mb) * C.K *
                                                                             (S.general_obs ? c.pauli_blocks : c.tiles * c.waves)));
  c.off_partF = off;   off = align_up(off + sizeof(float) * std::max<int64_t>(1, int64_t(c.mb) * c.partF_seg_floats));
  c.off_Gr = off;      off = align_up(off + sizeof(float) * std::max<int64_t>(1, int64_t(c.mb) * c.n_angle));
  c.ws_bytes = off;
  return QF_OK;
}

// The observables as Pauli records in the bit order of the state they are
// applied to: logical for the per-gate paths, the last pass's output order for
// the fused path.
inline std::vector<PauliRec> pauli_table(const PlanCore& c) {
  std::vector<PauliRec> out;
  for (const qf_pauli& o : c.C.obs) {
    PauliRec r{0, 0, 0, 0};
    for (int q = 0; q < c.C.n; ++q) {
      const int m = (!c.per_gate && !c.S.final_map.empty()) ? c.S.final_map[q] : q;
      if ((o.x_mask >> q) & 1) r.xm |= 1u << m;
      if ((o.z_mask >> q) & 1) r.zm |= 1u << m;
    }
    r.ny = __builtin_popcountll(o.x_mask & o.z_mask) & 3;
    out.push_back(r);
  }
  return out;
}

template <class T>
inline T* at(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

// ---------------------------------------------------------------- per-gate baseline
// One kernel launch per gate: the forward reads and writes the whole state for
// every gate; the backward reads psi and lambda and writes both back for every
// gate (un-applying it), plus the gate's functional partial sums.  This is the
// unfused reference point for the fused passes (Sec. 3.1: every gate touches
// O(2^n) amplitudes).
// Real is float on the baseline and double on the complex128 validation path.
template <class Real, class Exec>
qf_status run_forward_pg(const PlanCore& c, Exec& ex, const Real* theta, const Real* x, Real* E, char* ws,
                         const Real* psi0 = nullptr) {
  const int64_t SA = 2 * c.amps;
  const Real* csh = at<Real>(ws, c.off_coef_sh);
  const Real* cps = at<Real>(ws, c.off_coef_ps);
  ex.pg_coef(theta, x, ws);
  for (int mb0 = 0; mb0 < c.B; mb0 += c.mb) {
    const int nb = std::min(c.mb, c.B - mb0);
    Real* psi = at<Real>(ws, c.off_ckpt) + int64_t(mb0) * SA;
    if (psi0) ex.pg_copy(psi, psi0 + int64_t(mb0) * SA, nb);
    else ex.pg_init(psi, nb);
    int r = 0;
    for (const qf_gate& g : c.C.gates) {
      if (g.kind == QF_CZ) ex.pg_cz(psi, (Real*)nullptr, nb, g.q0, g.q1);
      else ex.pg_rot(psi, nb, mb0, r++, csh, cps);
    }
    ex.pauli_expect((const Real*)psi, SA, nb, at<Real>(ws, c.off_partE));
    ex.pauli_reduce_E(nb, mb0, (const Real*)at<Real>(ws, c.off_partE), E);
  }
  return ex.status();
}

template <class Real, class Exec>
qf_status run_backward_pg(const PlanCore& c, Exec& ex, const Real* theta, const Real* x, const Real* dE,
                          Real* dtheta, Real* dx, char* ws) {
  const int64_t SA = 2 * c.amps;
  const Real* csh = at<Real>(ws, c.off_coef_sh);
  const Real* cps = at<Real>(ws, c.off_coef_ps);
  Real* partF = at<Real>(ws, c.off_partF);
  Real* Gr = at<Real>(ws, c.off_Gr);
  const int nrot = c.n_angle;
  for (int mb0 = 0; mb0 < c.B; mb0 += c.mb) {
    const int nb = std::min(c.mb, c.B - mb0);
    const Real* fin = at<Real>(ws, c.off_ckpt) + int64_t(mb0) * SA;
    Real* psi = at<Real>(ws, c.off_lam);
    Real* lam = psi + SA * nb;
    ex.pg_copy(psi, fin, nb);
    ex.pauli_seed((const Real*)psi, SA, lam, SA, nb, mb0, dE);
    int r = nrot;
    for (int64_t j = (int64_t)c.C.gates.size() - 1; j >= 0; --j) {
      const qf_gate& g = c.C.gates[j];
      if (g.kind == QF_CZ) {
        ex.pg_cz(psi, lam, nb, g.q0, g.q1);
        continue;
      }
      --r;
      ex.pg_rot_bwd(psi, lam, nb, mb0, r, r % c.pg_chunk, csh, cps, partF);
      if (r % c.pg_chunk == 0) {
        const int cnt = std::min(c.pg_chunk, nrot - r);
        ex.pg_assemble(r, cnt, nb, mb0, theta, x, (const Real*)partF, Gr);
      }
    }
    ex.pg_reduce_grads(nb, mb0, (const Real*)Gr, dtheta, dx, mb0 > 0);
  }
  return ex.status();
}

// ---------------------------------------------------------------- fused path
// Runs the forward passes of one micro-batch; returns the final state and its
// per-sample stride (floats).
template <class Exec>
std::pair<const float*, int64_t> forward_passes(const PlanCore& c, Exec& ex, char* ws, int mb0, int nb,
                                                bool keep_ckpt, float* ckpt_base, bool do_expect,
                                                const float* psi0) {
  const int64_t SA = 2 * c.amps;   // floats per state
  float* work = at<float>(ws, c.off_work);
  float* partE = at<float>(ws, c.off_partE);
  const float* src = nullptr;
  int64_t src_stride = 0;
  for (int p = 0; p < c.P; ++p) {
    const int s = p / c.ckpt;
    const bool seg_end = (p == c.seg_begin[s + 1] - 1);
    PassLaunch L;
    L.pass = p;
    L.nb = nb;
    L.sample0 = mb0;
    L.src0 = src;
    L.src0_stride = src_stride;
    if (p == 0 && psi0) {   // a given initial state, logical order
      L.src0 = psi0 + int64_t(mb0) * SA;
      L.src0_stride = SA;
      L.load_input = true;
    }
    if (keep_ckpt && seg_end) {
      L.dst = ckpt_base + s * SA;
      L.dst_stride = SA * c.n_seg;
    } else {
      L.dst = work + (p & 1) * SA * nb;
      L.dst_stride = SA;
    }
    L.partE = partE;
    L.do_expect = (do_expect && p == c.P - 1) ? 1 : 0;
    ex.pass(L);
    src = L.dst;
    src_stride = L.dst_stride;
  }
  return {src, src_stride};
}

template <class Exec>
qf_status run_forward_fused(const PlanCore& c, Exec& ex, const float* theta, const float* x, float* E, char* ws,
                            const float* psi0 = nullptr) {
  const int64_t SA = 2 * c.amps;
  ex.coef(theta, x, ws);
  for (int mb0 = 0; mb0 < c.B; mb0 += c.mb) {
    const int nb = std::min(c.mb, c.B - mb0);
    float* ck = at<float>(ws, c.off_ckpt) + (c.store ? int64_t(mb0) * c.n_seg * SA : 0);
    const auto fin = forward_passes(c, ex, ws, mb0, nb, c.store != 0, ck, true, psi0);
    if (c.S.general_obs) {
      // X / Y observables: from the stored output state, in its bit order
      ex.pauli_expect(fin.first, fin.second, nb, at<float>(ws, c.off_partE));
      ex.pauli_reduce_E(nb, mb0, (const float*)at<float>(ws, c.off_partE), E);
    } else {
      ex.reduce_E(nb, mb0, at<float>(ws, c.off_partE), E);
    }
  }
  return ex.status();
}

template <class Exec>
qf_status run_backward_fused(const PlanCore& c, Exec& ex, const float* theta, const float* x, const float* dE,
                             float* dtheta, float* dx, char* ws, const float* psi0 = nullptr) {
  const int64_t SA = 2 * c.amps;
  const int64_t SS = c.memsave ? c.amps : SA;   // words per stored pass output
  const bool bf = c.memsave != 0;
  float* seg = at<float>(ws, c.off_seg);
  float* work = at<float>(ws, c.off_work);
  float* lam = at<float>(ws, c.off_lam);
  float* partF = at<float>(ws, c.off_partF);
  float* Gr = at<float>(ws, c.off_Gr);
  for (int mb0 = 0; mb0 < c.B; mb0 += c.mb) {
    const int nb = std::min(c.mb, c.B - mb0);
    float* ck = at<float>(ws, c.off_ckpt) + (c.store ? int64_t(mb0) * c.n_seg * SA : 0);
    if (!c.store) forward_passes(c, ex, ws, mb0, nb, true, ck, false, psi0);
    const int64_t ck_stride = SA * c.n_seg;
    int li = 0;
    for (int s = c.n_seg - 1; s >= 0; --s) {
      const int a = c.seg_begin[s], b = c.seg_begin[s + 1];
      // recompute the segment, storing every pass output but the last (in the
      // uncompute mode the adjoint passes rebuild psi instead, from the
      // segment's checkpointed output through the work states)
      for (int p = a; p <= b - 2 && !c.uncompute; ++p) {
        PassLaunch L;
        L.pass = p;
        L.nb = nb;
        L.sample0 = mb0;
        if (p == a) {
          if (s > 0) { L.src0 = ck + (s - 1) * SA; L.src0_stride = ck_stride; }
          else if (psi0) { L.src0 = psi0 + int64_t(mb0) * SA; L.src0_stride = SA; L.load_input = true; }
        } else if (bf) {
          // the recompute continues from the float32 output of the previous pass
          L.src0 = work + ((p - 1) & 1) * SA * nb;
          L.src0_stride = SA;
        } else {
          L.src0 = seg + int64_t(p - 1 - a) * SA;
          L.src0_stride = SA * (c.ckpt - 1);
        }
        if (bf) {
          // float32 output for the next recompute pass, bfloat16 copy kept for the adjoint pass
          L.dst = work + (p & 1) * SA * nb;
          L.dst_stride = SA;
          L.dst2 = reinterpret_cast<uint32_t*>(seg) + int64_t(p - a) * SS;
          L.dst2_stride = SS * (c.ckpt - 1);
        } else {
          L.dst = seg + int64_t(p - a) * SA;
          L.dst_stride = SA * (c.ckpt - 1);
        }
        ex.pass(L);
      }
      // fused adjoint passes
      for (int p = b - 1; p >= a; --p) {
        PassLaunch L;
        L.pass = p;
        L.bwd = true;
        L.nb = nb;
        L.sample0 = mb0;
        if (p == b - 1) { L.src0 = ck + s * SA; L.src0_stride = ck_stride; }
        else if (c.uncompute) { L.src0 = work + (p & 1) * SA * nb; L.src0_stride = SA; }
        else { L.src0 = seg + int64_t(p - a) * SS; L.src0_stride = SS * (c.ckpt - 1); L.src0_bf16 = bf; }
        if (p == c.P - 1 && c.S.general_obs)   // seed from the stored output state
          ex.pauli_seed((const float*)(ck + s * SA), ck_stride, lam + li * SA * nb, SA, nb, mb0, dE);
        if (p != c.P - 1 || c.S.general_obs) { L.src1 = lam + li * SA * nb; L.src1_stride = SA; }
        if (p > 0) { L.dst = lam + (1 - li) * SA * nb; L.dst_stride = SA; }
        if (c.uncompute && p > a) { L.dpsi = work + ((p - 1) & 1) * SA * nb; L.dpsi_stride = SA; }
        L.partF = partF + int64_t(nb) * c.partF_off[p];
        L.dE = dE;
        ex.pass(L);
        li = 1 - li;
      }
      ex.assemble(s, nb, mb0, theta, x, partF, Gr);
    }
    ex.reduce_grads(nb, mb0, Gr, dtheta, dx, mb0 > 0);
  }
  return ex.status();
}

// psi0: the initial states of the batch (complex64, logical order), or null
// for |0...0>; the backward needs the same psi0 as the forward.
template <class Exec>
qf_status run_forward(const PlanCore& c, Exec& ex, const float* theta, const float* x, float* E, char* ws,
                      const float* psi0 = nullptr) {
  if (c.per_gate) return run_forward_pg(c, ex, theta, x, E, ws, psi0);
  return run_forward_fused(c, ex, theta, x, E, ws, psi0);
}

template <class Exec>
qf_status run_backward(const PlanCore& c, Exec& ex, const float* theta, const float* x, const float* dE,
                       float* dtheta, float* dx, char* ws, const float* psi0 = nullptr) {
  if (c.per_gate) return run_backward_pg(c, ex, theta, x, dE, dtheta, dx, ws);
  return run_backward_fused(c, ex, theta, x, dE, dtheta, dx, ws, psi0);
}

}  // namespace qf
