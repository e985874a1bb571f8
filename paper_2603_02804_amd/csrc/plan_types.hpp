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
constexpr int kSwizzleBits = 4;    // LDS XOR swizzle folds 4-bit chunks

enum OpKind : int32_t {
  OP_INIT0 = 1,   // a=layout: |0...0> restricted to the tile
  OP_LOAD = 2,    // a=layout, b=buffer (0 psi, 1 lambda), c=map (0 in, 1 out)
  OP_STORE = 3,   // a=layout, b=buffer (0 = destination), c=map
  OP_PERM = 4,    // a=from layout, b=to layout (psi, and lambda in the backward)
  OP_U2 = 5,      // a=register bit, b=coefficient ref (>=0 shared, <0 per-sample -1-idx)
  OP_U2ADJ = 6,   // same, applies u^dagger to psi and lambda
  OP_CZ = 7,      // a=layout, b=first CZ group, c=number of groups
  OP_EXPECT = 8,  // a=layout: Z-string expectations of psi -> partial sums
  OP_SEED = 9,    // a=layout: lambda = 2 sum_k g_k O_k psi
  OP_FUNC = 10,   // a=entries, b=first FuncEntry: Im<lambda|P_q|psi> for P=X,Y,Z
};

struct Op {
  int32_t kind, a, b, c;
};

// Uniform address tables of one layout.  Index of the amplitude held by thread
// t in register slot jj:  T(t) ^ reg[jj] where T(t) = XOR of thr[i] over the set
// bits i of t.  Three index spaces: LDS element (XOR-swizzled), logical basis
// index (qubit q at bit q) and memory index (only for load / store layouts).
struct LayoutRec {
  uint32_t lds_reg[1 << kMaxR];
  uint32_t lds_thr[kMaxThreadBits];
  uint32_t log_reg[1 << kMaxR];
  uint32_t log_thr[kMaxThreadBits];
  uint32_t mem_reg[1 << kMaxR];
  uint32_t mem_thr[kMaxThreadBits];
  int32_t reg_qubit[kMaxR];   // logical qubit in register bit j (-1: none)
  int32_t pad[3];
};

// CZ gates between qubits i and i+shift for every set bit i of mask.
struct CzGroup {
  uint32_t shift, mask;
};

struct FuncEntry {
  int32_t regbit, slot;
};

// Per-pass tile mapping.  Tile id bit i selects the value of the i-th non-local
// qubit: logical bit nl_log[i], memory bit nl_in[i] before the pass and
// nl_out[i] after it.
struct PassRec {
  int32_t fop_begin, fop_count;   // forward program
  int32_t bop_begin, bop_count;   // backward program
  int32_t n_nonlocal;
  int32_t n_slots;                // fused runs whose functionals the backward writes
  int32_t pad[2];
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
