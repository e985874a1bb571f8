// plan_types.hpp -- plain-old-data records that the host planner writes and the
// pass kernels read.  Shared by the planner, the HIP kernels and the CPU
// schedule checker; nothing here is shared with the oracle.
//
// A fused pass processes one tile of 2^k amplitudes of one sample per workgroup.
// Inside the workgroup every lane holds 2^R amplitudes in registers; the tile's
// k "tile positions" are split between R register bits and log2(threads) thread
// bits by a *layout*.  Gates act only on register bits; a PERM op moves the tile
// through LDS into another layout (swap-to-local inside the tile).  Which logical
// qubit sits at which tile position, and which memory bit holds which qubit
// before and after the pass, are fixed per pass by the planner.
#pragma once
#include <stdint.h>

namespace qf {

constexpr int kMaxR = 5;           // register-resident qubits per lane
constexpr int kMaxThreadBits = 8;  // up to 256 threads per workgroup
constexpr int kMaxTileQubits = kMaxR + kMaxThreadBits;
constexpr int kMaxQubits = 30;
constexpr int kDefaultTileQubits = 12;
constexpr int kDefaultRegQubits = 4;

// Ops of a pass program.  Every run (merged single-qubit rotations of one
// qubit) is split as RZ(a) RY(b) RZ(c): only the real RY(b) touches amplitude
// pairs; the RZ phases and the CZ signs are diagonal and are applied where they
// are cheapest.  While all their qubits are held in thread bits (or are outside
// the tile) they reduce to one complex factor per thread, accumulated in a
// pending per-thread phase that is multiplied into the amplitudes at the next
// PERM or STORE.  Otherwise they are applied per amplitude (CZA, PHASEA).
enum OpKind : int32_t {
  OP_INIT0 = 1,   // a=layout: |0...0> restricted to the tile
  OP_LOAD = 2,    // a=layout, b=buffer (0 psi, 1 lambda), c=map (0 in, 1 out)
  OP_STORE = 3,   // a=layout, c=map: flush the pending phase, write psi (fwd) / lambda (bwd)
  OP_PERM = 4,    // a=from layout, b=to layout: flush the pending phase, exchange through LDS
  OP_RY = 5,      // a=register bit, b=run coefficient ref (>=0 shared, <0 per-sample -1-idx),
                  // c=run id; backward: RY(b)^dagger on psi and lambda
  OP_DIAGT = 6,   // a=layout, b=first CZ group, c=groups, d=first phase event, e=events:
                  // diagonal gates on thread-held qubits, folded into the pending phase
  OP_CZA = 7,     // a=CzaRec, b=layout: CZ signs for edges touching register bits
  OP_PHASEA = 8,  // a=register bit, b=phase event: RZ phase on a register-held qubit
  OP_EXPECT = 9,  // a=layout: Z-string expectations of psi -> partial sums
  OP_SEED = 10,   // a=layout: lambda = 2 sum_k g_k O_k psi
  OP_FUNC = 11,   // a=R entries, b=first FuncEntry (entry j: register bit j, slot or -1):
                  // Im<lambda|P_q|psi> for P=X,Y,Z
  OP_RYG = 12,    // a=entries, b=first RygEntry, c=mask of their register bits: the RY of
                  // several runs on distinct register bits (they commute), bits ascending
  OP_EPOCH = 13,  // a=first EpochRec, b=count: consecutive register epochs (PERM, DIAGT,
                  // PHASEA*, CZA, RY group forward; FUNC, RY group, CZA, PHASEA*, DIAGT,
                  // PERM backward), one loop iteration each
};

struct Op {
  int32_t kind, a, b, c, d, e, f, g;
};

// RZ phase on qubit q: amplitudes with bit q = 0 gain w, bit q = 1 gain conj(w);
// w = e^{-i a_prev/2} e^{-i c_next/2} joins the trailing RZ of one run with the
// leading RZ of the next run on the same qubit (only diagonal gates between).
struct PhaseEv {
  int32_t q;
  int32_t ref;    // event coefficient: >=0 shared row, <0 per-sample row -1-idx
};

// A Pauli-string observable i^ny X^xm Z^zm (Y where both masks are set; ny =
// number of Y factors mod 4), masks in the bit order of the state it is applied
// to: (P psi)_y = i^ny (-1)^{popcount((y ^ xm) & zm)} psi_{y ^ xm} (App. B.2).
struct PauliRec {
  uint32_t xm, zm;
  int32_t ny;
  int32_t pad;
};

// Per-amplitude CZ signs on a register layout: sign(jj) = bit jj of sr XOR
// parity over register bits j set in jj of parity(A & cmask[j]), A = the
// thread's logical base index (thread and tile bits).
struct CzaRec {
  uint32_t sr;
  uint32_t cmask[kMaxR];
  uint32_t pad[2];
};

// Phase event definition for the coefficient kernel: w = u_a(prev) * u_c(next).
struct EventRec {
  int32_t prev_ref;   // coefficient ref of the run before (or INT32_MIN: none)
  int32_t next_ref;   // coefficient ref of the run after (or INT32_MIN: none)
  int32_t per_sample;
  int32_t pad;
};

// Uniform address data of one layout.  Index of the amplitude held by thread
// t in register slot jj:  T(t) ^ J(jj), with T(t) = XOR of thr[i] over the set
// bits i of t and J(jj) = XOR of reg[j] over the set bits j of jj.  Three index
// spaces: LDS byte offset (XOR-swizzled element index times kLdsElemBytes, so
// that the XOR is the address), logical basis index (qubit q at bit q) and
// memory index (only for load / store layouts).
constexpr uint32_t kLdsElemBytes = 8;   // one complex64 amplitude
struct LayoutRec {
  uint32_t lds_reg[kMaxR];
  uint32_t lds_thr[kMaxThreadBits];
  uint32_t log_reg[kMaxR];
  uint32_t log_thr[kMaxThreadBits];
  uint32_t mem_reg[kMaxR];
  uint32_t mem_thr[kMaxThreadBits];
  int32_t reg_qubit[kMaxR];
  int32_t pad[1];
};

// Thread part of a layout's three indices for one thread: the XOR of lds_thr,
// log_thr and mem_thr over the set bits of the thread id.
struct ThrBase {
  uint32_t lds, log, mem, pad;
};

// XOR of per-bit contributions over the set bits of jj.
inline uint32_t reg_index(const uint32_t* per_bit, int jj) {
  uint32_t v = 0;
  for (int j = 0; j < kMaxR; ++j)
    if ((jj >> j) & 1) v ^= per_bit[j];
  return v;
}

// CZ gates between qubits i and i+shift for every set bit i of mask.
struct CzGroup {
  uint32_t shift, mask;
};

struct FuncEntry {
  int32_t regbit, slot;
};

// One run of an OP_RYG group: its register bit and coefficient ref.
struct RygEntry {
  int32_t regbit, ref;
};

// PHASEA inside an epoch: register bit and phase event.
struct PhaEntry {
  int32_t regbit, pev;
};

// The sub-ops of one epoch; -1 / 0 fields mark sub-ops that are absent.  At
// most kEpochMaxPhaseA PHASEA sub-ops (epochs with more stay unfused; they are
// diagonal, so their order within the epoch does not matter).
constexpr int kEpochMaxPhaseA = 8;
struct EpochRec {
  int32_t perm_from, perm_to;                          // PERM (from -1: none)
  int32_t diag_layout, czg_first, czg_count, pev_first, pev_count;   // DIAGT (layout -1: none)
  int32_t pha_first, pha_count;                        // PhaEntry range
  int32_t cza, cza_layout;                             // CZA (-1: none)
  int32_t ry_kind, ry_a, ry_b;                         // run group: first RygEntry a, bit mask b (0: none)
  int32_t func_count, func_first, func_full;           // FUNC (backward; func_full unused)
  int32_t pad;
};

// Per-pass tile mapping.  Tile id bit i selects the value of the i-th non-local
// qubit: logical bit nl_log[i], memory bit nl_in[i] before the pass and
// nl_out[i] after it.
struct PassRec {
  int32_t fop_begin, fop_count;   // forward program
  int32_t bop_begin, bop_count;   // backward program
  int32_t n_nonlocal;
  int32_t n_slots;                // fused runs whose functionals the backward writes
  int32_t fload_begin;            // pass 0: forward program that loads a caller's initial
                                  // state (logical order) instead of generating |0...0>; -1
  int32_t pad;
  uint8_t nl_log[32], nl_in[32], nl_out[32];
};

// One fused run: consecutive single-qubit rotations on one qubit.
struct RunRec {
  int32_t q;
  int32_t gate_begin, gate_count;   // into the run-gate list (forward order)
  int32_t coef;                     // >=0 shared coefficient row, <0 per-sample row -1-idx
  int32_t pass, slot;               // where the backward computes its functionals
  int32_t pad[2];
};

// Gate data needed on the device for coefficients and gradient assembly.
struct GateRec {
  int32_t kind;        // 0 RX, 1 RY, 2 RZ
  int32_t theta_idx;   // or -1
  int32_t input_idx;   // or -1
  int32_t out_idx;     // column in the per-sample gradient table
};

}  // namespace qf
