// plan.hpp -- host planner: gate list -> fused pass schedule.
//
// Forward fusion (Sec. 3.2): consecutive single-qubit rotations on one qubit are
// merged into one 2x2 "run"; a pass applies every run and CZ that is ready and
// whose qubit is local to the pass's tile, reading and writing the state once.
// Backward fusion (Sec. 3.3): each pass has a mirrored program that starts from
// the stored pass output and the adjoint state, and for every run, in reverse
// order, evaluates the functionals that give the run's gradients and un-applies
// the run from both states in registers.  CZ gates are real and self-adjoint, so
// the same sign operation serves both directions (App. B.1).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "plan_types.hpp"
#include "qfuse.h"

namespace qf {

struct Circuit {
  int n = 0, P = 0, F = 0, K = 0;
  std::vector<qf_gate> gates;       // CNOT lowered (see circuit_from_desc)
  std::vector<qf_pauli> obs;
  std::vector<double> consts;       // fixed angles of internal gates: theta_idx = -2 - index
};

// Internal gate with a fixed angle: theta_idx encodes the constant's index.
inline bool gate_is_const(const qf_gate& g) { return g.theta_idx <= -2; }

// Copies a validated description.  CNOT(c, t) becomes RY_t(-pi/2), CZ(c, t),
// RY_t(pi/2) (since H = RY(pi/2) Z and Z commutes with CZ, H CZ H = CNOT), so
// that the planner fuses it like any rotation and diagonal gate.
void circuit_from_desc(const qf_circuit_desc* d, Circuit* C);

// Returns QF_OK or a status with a message; checks every index and size.
qf_status validate_circuit(const qf_circuit_desc* d, std::string* msg);

struct Tuning {
  int mode = 0;          // 0 fused, 1 per-gate
  int k = 0;             // tile qubits
  int R = 0;             // register qubits
  int fusion = 0;        // runs per qubit per pass
  int ckpt = 0;          // passes per checkpoint segment
  int micro = 0;         // samples per micro-batch
  int store = -1;        // keep checkpoints of the whole batch in the forward
  int memsave = 0;       // stored pass outputs of the active segment as bfloat16 pairs
  int uncompute = 0;     // the adjoint passes rebuild psi; no recompute (1: on)
  int fill = 0;          // end-of-pass epochs with fewer runs wait (0: R, -1: none)
};

struct Schedule {
  int n = 0, k = 0, R = 0, NT = 0, active = 0, tiles_log2 = 0, thread_bits = 0;
  int fusion = 0;
  int fill = 0;                       // end-of-pass epochs with fewer runs wait for the next pass
  std::vector<RunRec> runs;
  std::vector<int32_t> run_gates;     // GateRec indices of each run, forward order
  std::vector<GateRec> gates;         // rotations in circuit order
  int n_coef_shared = 0, n_coef_ps = 0;
  std::vector<PassRec> passes;
  std::vector<Op> ops;
  std::vector<LayoutRec> layouts;
  std::vector<CzGroup> czg;
  std::vector<FuncEntry> funcs;
  std::vector<RygEntry> rygs;
  std::vector<EpochRec> epochs;
  std::vector<PhaEntry> phas;
  std::vector<EventRec> events;       // phase event coefficient definitions
  int n_ev_shared = 0, n_ev_ps = 0;
  std::vector<PhaseEv> pev;           // phase events referenced by DIAGT / PHASEA ops
  std::vector<CzaRec> cza;
  std::vector<int32_t> pass_run_begin, pass_runs;   // runs of each pass, slot order
  // observables with X or Y parts: the last pass stores the full output state
  // (trailing diagonal gates applied) in memory bit order final_map[qubit], and
  // separate kernels form E and the adjoint seed from it
  bool general_obs = false;
  std::vector<int32_t> final_map;
  int max_slots = 0;
  // per-sample op counts over all forward passes
  int64_t n_perm = 0, n_u2 = 0, n_cz = 0;
  int64_t n_diag_thread = 0, n_diag_amp = 0;   // diagonal items folded per thread / applied per amplitude
};

// Fused schedule.  Fails only on internal inconsistencies (the circuit is
// validated before).
bool build_schedule(const Circuit& c, const Tuning& t, Schedule* s, std::string* msg);

// Runs and gate tables only, one run per rotation gate (the per-gate baseline).
void build_gate_runs(const Circuit& c, Schedule* s);

// Swizzled LDS element index of tile index i: tile bits 5..11 each add a
// pattern to element bits 0..4 (the 32 eight-byte bank slots that one LDS cycle
// serves), chosen so that almost every set of 8 tile positions (a 256-thread
// layout's thread positions) holds 5 positions independent on those bits: the
// lanes 0..4 of every layout then reach 32 distinct bank slots.
inline uint32_t lds_swizzle(uint32_t i) {
  constexpr uint32_t fold[7] = {13u, 21u, 25u, 19u, 31u, 22u, 7u};
  uint32_t f = 0;
  for (int b = 0; b < 7; ++b)
    if ((i >> (5 + b)) & 1u) f ^= fold[b];
  return i ^ f;
}

}  // namespace qf
