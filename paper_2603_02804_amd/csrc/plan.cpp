// plan.cpp -- fused pass scheduler (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <map>
#include <numeric>

namespace qf {

qf_status validate_circuit(const qf_circuit_desc* d, std::string* msg) {
  auto fail = [&](qf_status s, const std::string& m) {
    if (msg) *msg = m;
    return s;
  };
  if (!d) return fail(QF_ERR_INVALID_ARG, "circuit description is NULL");
  if (d->n_qubits < 1 || d->n_qubits > kMaxQubits)
    return fail(QF_ERR_UNSUPPORTED, "n_qubits must be in [1, 30]");
  if (d->n_params < 0 || d->n_inputs < 0 || d->n_gates < 0 || d->n_obs < 0)
    return fail(QF_ERR_INVALID_ARG, "negative size");
  if (d->n_gates > 0 && !d->gates) return fail(QF_ERR_INVALID_ARG, "gates is NULL");
  if (d->n_obs > 0 && !d->obs) return fail(QF_ERR_INVALID_ARG, "obs is NULL");
  if (d->n_obs > 64) return fail(QF_ERR_UNSUPPORTED, "at most 64 observables");
  const int n = d->n_qubits;
  for (int64_t j = 0; j < d->n_gates; ++j) {
    const qf_gate& g = d->gates[j];
    const std::string at = " (gate " + std::to_string(j) + ")";
    if (g.kind < QF_RX || g.kind > QF_CNOT) return fail(QF_ERR_INVALID_ARG, "unknown gate kind" + at);
    if (g.q0 < 0 || g.q0 >= n) return fail(QF_ERR_INVALID_ARG, "qubit out of range" + at);
    if (g.kind == QF_CZ || g.kind == QF_CNOT) {
      if (g.q1 < 0 || g.q1 >= n) return fail(QF_ERR_INVALID_ARG, "two-qubit gate partner out of range" + at);
      if (g.q1 == g.q0) return fail(QF_ERR_INVALID_ARG, "two-qubit gate on a single qubit" + at);
      if (g.theta_idx != -1 || g.input_idx != -1)
        return fail(QF_ERR_INVALID_ARG, "CZ and CNOT carry no angle" + at);
    } else {
      if ((g.theta_idx >= 0) == (g.input_idx >= 0))
        return fail(QF_ERR_INVALID_ARG, "rotation needs exactly one angle source" + at);
      if (g.theta_idx >= d->n_params) return fail(QF_ERR_INVALID_ARG, "theta_idx out of range" + at);
      if (g.input_idx >= d->n_inputs) return fail(QF_ERR_INVALID_ARG, "input_idx out of range" + at);
      if (g.theta_idx < -1 || g.input_idx < -1) return fail(QF_ERR_INVALID_ARG, "bad angle index" + at);
    }
  }
  for (int k = 0; k < d->n_obs; ++k) {
    const uint64_t lim = (n == 64) ? ~0ull : ((1ull << n) - 1);
    if ((d->obs[k].x_mask | d->obs[k].z_mask) & ~lim)
      return fail(QF_ERR_INVALID_ARG, "observable acts outside the register");
  }
  return QF_OK;
}

void circuit_from_desc(const qf_circuit_desc* d, Circuit* C) {
  C->n = d->n_qubits;
  C->P = d->n_params;
  C->F = d->n_inputs;
  C->K = d->n_obs;
  C->gates.clear();
  C->consts.clear();
  C->obs.assign(d->obs, d->obs + d->n_obs);
  const double half_pi = 1.5707963267948966;
  for (int64_t j = 0; j < d->n_gates; ++j) {
    const qf_gate& g = d->gates[j];
    if (g.kind != QF_CNOT) {
      C->gates.push_back(g);
      continue;
    }
    const int t = g.q1;
    C->consts.push_back(-half_pi);
    C->gates.push_back({QF_RY, t, -1, -1 - (int)C->consts.size(), -1});
    C->gates.push_back({QF_CZ, g.q0, t, -1, -1});
    C->consts.push_back(half_pi);
    C->gates.push_back({QF_RY, t, -1, -1 - (int)C->consts.size(), -1});
  }
}

namespace {

struct Unit {
  int kind;   // 0 run, 1 cz
  int a, b;   // run: a = qubit; cz: qubits
  int run;    // run id
  int order;  // index of the unit's first gate in the circuit
};

struct Builder {
  const Circuit& C;
  Schedule& S;
  int n, k, R, tb, F;
  std::vector<Unit> units;
  std::vector<std::vector<int>> wire;
  std::vector<size_t> ptr;
  std::vector<int> depth;
  int64_t remaining = 0;
  int64_t max_runs_per_pass = 0;

  Builder(const Circuit& c, Schedule& s) : C(c), S(s) {}

  int front(int q) const { return ptr[q] < wire[q].size() ? wire[q][ptr[q]] : -1; }
  bool ready(int u) const {
    const Unit& U = units[u];
    if (U.kind == 0) return front(U.a) == u;
    return front(U.a) == u && front(U.b) == u;
  }
  void finish(int u) {
    const Unit& U = units[u];
    ptr[U.a]++;
    if (U.kind == 1) ptr[U.b]++;
    else depth[U.a]++;
    remaining--;
  }
};

void build_runs(const Circuit& C, Schedule& S, std::vector<Unit>* units,
                std::vector<std::vector<int>>* wire, bool one_gate_per_run) {
  const int n = C.n;
  std::vector<std::vector<int32_t>> run_lists;
  std::vector<int> open(n, -1);
  std::vector<int> run_q;
  if (units) units->clear();
  if (wire) wire->assign(n, {});
  S.gates.clear();
  int order = 0;
  for (const qf_gate& g : C.gates) {
    ++order;
    if (g.kind == QF_CZ) {
      if (units) {
        int u = (int)units->size();
        units->push_back({1, g.q0, g.q1, -1, order});
        (*wire)[g.q0].push_back(u);
        (*wire)[g.q1].push_back(u);
      }
      open[g.q0] = open[g.q1] = -1;
      continue;
    }
    int gi = (int)S.gates.size();
    S.gates.push_back({g.kind, g.theta_idx, g.input_idx, gi});
    int r = one_gate_per_run ? -1 : open[g.q0];
    if (r < 0) {
      r = (int)run_lists.size();
      run_lists.emplace_back();
      run_q.push_back(g.q0);
      if (units) {
        int u = (int)units->size();
        units->push_back({0, g.q0, -1, r, order});
        (*wire)[g.q0].push_back(u);
      }
      open[g.q0] = r;
    }
    run_lists[r].push_back(gi);
  }
  S.runs.assign(run_lists.size(), RunRec{});
  S.run_gates.clear();
  S.n_coef_shared = S.n_coef_ps = 0;
  for (size_t r = 0; r < run_lists.size(); ++r) {
    RunRec& rr = S.runs[r];
    rr.q = run_q[r];
    rr.gate_begin = (int)S.run_gates.size();
    rr.gate_count = (int)run_lists[r].size();
    bool ps = false;
    for (int gi : run_lists[r]) {
      S.run_gates.push_back(gi);
      ps = ps || S.gates[gi].input_idx >= 0;
    }
    rr.coef = ps ? -1 - (S.n_coef_ps++) : (S.n_coef_shared++);
    rr.pass = rr.slot = -1;
  }
}

LayoutRec make_layout(const std::vector<int>& reg_pos, const std::vector<int>& thr_pos,
                      const std::vector<int>& local, const std::vector<int>* map, int R) {
  LayoutRec L;
  std::memset(&L, 0, sizeof(L));
  for (int j = 0; j < kMaxR; ++j) {
    L.reg_qubit[j] = (j < R) ? local[reg_pos[j]] : -1;
    if (j >= R) continue;
    L.lds_reg[j] = lds_swizzle(1u << reg_pos[j]) * kLdsElemBytes;
    L.log_reg[j] = 1u << local[reg_pos[j]];
    L.mem_reg[j] = map ? (1u << (*map)[local[reg_pos[j]]]) : 0u;
  }
  for (size_t b = 0; b < thr_pos.size(); ++b) {
    L.lds_thr[b] = lds_swizzle(1u << thr_pos[b]) * kLdsElemBytes;
    L.log_thr[b] = 1u << local[thr_pos[b]];
    L.mem_thr[b] = map ? (1u << (*map)[local[thr_pos[b]]]) : 0u;
  }
  return L;
}

// Orders thread positions so that the lanes of one LDS cycle reach distinct
// bank slots: lanes 0..4 take positions whose swizzled elements are independent
// on element bits 0..4 (32 lanes of 8-byte accesses in 256 bytes), lanes 0..3 if
// possible also on bits 0..3 (16 lanes in 128 bytes).  Greedy in tile order; the
// other positions follow in tile order.
std::vector<int> order_thread_positions(std::vector<int> free_pos, int tb) {
  std::vector<int> out;
  uint32_t b4[4] = {0, 0, 0, 0}, b5[5] = {0, 0, 0, 0, 0};   // reduced vectors by leading bit
  auto reduce = [](const uint32_t* basis, int bits, uint32_t v) {
    v &= (1u << bits) - 1u;
    for (int b = bits - 1; b >= 0; --b)
      if (((v >> b) & 1u) && basis[b]) v ^= basis[b];
    return v;
  };
  auto insert = [&](uint32_t* basis, int bits, uint32_t v) {
    v = reduce(basis, bits, v);
    for (int b = bits - 1; b >= 0; --b)
      if ((v >> b) & 1u) { basis[b] = v; return; }
  };
  while ((int)out.size() < std::min(tb, 5)) {
    int pick = -1, best = 0;
    for (size_t i = 0; i < free_pos.size() && best < 2; ++i) {
      const uint32_t e = lds_swizzle(1u << free_pos[i]);
      const int score = reduce(b5, 5, e) == 0 ? 0 : (out.size() < 4 && reduce(b4, 4, e) != 0) || out.size() >= 4 ? 2 : 1;
      if (score > best) { best = score; pick = (int)i; }
    }
    if (pick < 0) break;
    const uint32_t e = lds_swizzle(1u << free_pos[pick]);
    insert(b4, 4, e);
    insert(b5, 5, e);
    out.push_back(free_pos[pick]);
    free_pos.erase(free_pos.begin() + pick);
  }
  for (int p : free_pos) out.push_back(p);
  out.resize(tb);
  return out;
}

}  // namespace

void build_gate_runs(const Circuit& c, Schedule* s) {
  build_runs(c, *s, nullptr, nullptr, true);
}

// Replaces every maximal sequence of consecutive RY ops on distinct register
// bits by one OP_RYG op (entries sorted by bit: the rotations commute), and marks
// FUNC ops whose entries are exactly register bits 0..R-1 in order.  The kernels
// apply a full group in straight-line code.
static void group_register_runs(Schedule* Sp) {
  Schedule& S = *Sp;
  std::vector<Op> out;
  out.reserve(S.ops.size());
  auto regroup = [&](int begin, int count, int* nb, int* nc) {
    *nb = (int)out.size();
    int i = begin;
    const int end = begin + count;
    while (i < end) {
      const Op& o = S.ops[i];
      if (o.kind != OP_RY) {
        out.push_back(o);
        ++i;
        continue;
      }
      int j = i;
      uint32_t bits = 0;
      while (j < end && S.ops[j].kind == OP_RY && !((bits >> S.ops[j].a) & 1)) {
        bits |= 1u << S.ops[j].a;
        ++j;
      }
      if (j - i == 1) {
        out.push_back(o);
      } else {
        std::vector<RygEntry> es;
        for (int m = i; m < j; ++m) es.push_back({S.ops[m].a, S.ops[m].b});
        std::sort(es.begin(), es.end(), [](const RygEntry& x, const RygEntry& y) { return x.regbit < y.regbit; });
        out.push_back({OP_RYG, (int)es.size(), (int)S.rygs.size(), (int)bits, 0, 0, 0, 0});
        S.rygs.insert(S.rygs.end(), es.begin(), es.end());
      }
      i = j;
    }
    *nc = (int)out.size() - *nb;
  };
  for (PassRec& pr : S.passes) {
    int b, c;
    regroup(pr.fop_begin, pr.fop_count, &b, &c);
    pr.fop_begin = b;
    pr.fop_count = c;
    regroup(pr.bop_begin, pr.bop_count, &b, &c);
    pr.bop_begin = b;
    pr.bop_count = c;
  }
  S.ops.swap(out);
}

// Folds each register epoch into one OP_EPOCH op.  Forward: a PERM, then
// optionally a DIAGT, PHASEA ops, a CZA and one RY / RYG, in that order.
// Backward: optionally a FUNC, one RY / RYG, a CZA, PHASEA ops and a DIAGT,
// ending with a PERM.  The sub-ops keep their order, so execution is unchanged;
// ops outside these patterns stay as they are.
static void fuse_epochs(Schedule* Sp) {
  Schedule& S = *Sp;
  std::vector<Op> out;
  out.reserve(S.ops.size());
  int cur_begin = 0;   // first op of the program being built (runs never cross programs)
  auto blank = []() {
    EpochRec e;
    std::memset(&e, 0, sizeof(e));
    e.perm_from = e.perm_to = e.diag_layout = e.cza = -1;
    return e;
  };
  auto take_ry = [&](const Op& o, EpochRec* e) {
    e->ry_kind = 2;
    if (o.kind == OP_RY) {   // a single run becomes a group of one
      e->ry_a = (int)S.rygs.size();
      e->ry_b = 1 << o.a;
      S.rygs.push_back({o.a, o.b});
    } else {
      e->ry_a = o.b;
      e->ry_b = o.c;
    }
  };
  auto take_phas = [&](int* j, int end, EpochRec* e) {
    e->pha_first = (int)S.phas.size();
    while (*j < end && S.ops[*j].kind == OP_PHASEA) {
      S.phas.push_back({S.ops[*j].a, S.ops[*j].b});
      ++*j;
    }
    e->pha_count = (int)S.phas.size() - e->pha_first;
  };
  auto take_diag = [&](const Op& o, EpochRec* e) {
    e->diag_layout = o.a; e->czg_first = o.b; e->czg_count = o.c; e->pev_first = o.d; e->pev_count = o.e;
  };
  // consecutive epochs share one OP_EPOCH op (records are contiguous)
  auto emit = [&](const EpochRec& e) {
    if (!out.empty() && out.back().kind == OP_EPOCH && out.back().a + out.back().b == (int)S.epochs.size() &&
        (int)out.size() > cur_begin)
      out.back().b++;
    else
      out.push_back({OP_EPOCH, (int)S.epochs.size(), 1, 0, 0, 0, 0, 0});
    S.epochs.push_back(e);
  };
  auto fwd = [&](int begin, int count, int* nb, int* nc) {
    *nb = (int)out.size();
    cur_begin = *nb;
    const int end = begin + count;
    int i = begin;
    while (i < end) {
      if (S.ops[i].kind != OP_PERM) { out.push_back(S.ops[i++]); continue; }
      EpochRec e = blank();
      e.perm_from = S.ops[i].a;
      e.perm_to = S.ops[i].b;
      int j = i + 1;
      if (j < end && S.ops[j].kind == OP_DIAGT) take_diag(S.ops[j++], &e);
      take_phas(&j, end, &e);
      if (e.pha_count > kEpochMaxPhaseA) {   // rare: leave this epoch's ops as they are
        S.phas.resize(e.pha_first);
        for (int q = i; q < j; ++q) out.push_back(S.ops[q]);
        i = j;
        continue;
      }
      if (j < end && S.ops[j].kind == OP_CZA) { e.cza = S.ops[j].a; e.cza_layout = S.ops[j].b; ++j; }
      if (j < end && (S.ops[j].kind == OP_RY || S.ops[j].kind == OP_RYG)) {
        take_ry(S.ops[j++], &e);
      } else {
        // no runs (the exchange into the store layout at the end of a pass): its ops
        // stay single, so the epoch loop never applies an empty run group (as the
        // adjoint program, which fuses from its runs, leaves them too)
        S.phas.resize(e.pha_first);
        for (int q = i; q < j; ++q) out.push_back(S.ops[q]);
        i = j;
        continue;
      }
      emit(e);
      i = j;
    }
    *nc = (int)out.size() - *nb;
  };
  auto bwd = [&](int begin, int count, int* nb, int* nc) {
    *nb = (int)out.size();
    cur_begin = *nb;
    const int end = begin + count;
    int i = begin;
    while (i < end) {
      const int k = S.ops[i].kind;
      if (k != OP_FUNC && k != OP_RY && k != OP_RYG) { out.push_back(S.ops[i++]); continue; }
      EpochRec e = blank();
      int j = i;
      if (S.ops[j].kind == OP_FUNC) {
        e.func_count = S.ops[j].a; e.func_first = S.ops[j].b; e.func_full = S.ops[j].c;
        ++j;
      }
      if (j < end && (S.ops[j].kind == OP_RY || S.ops[j].kind == OP_RYG)) take_ry(S.ops[j++], &e);
      if (j < end && S.ops[j].kind == OP_CZA) { e.cza = S.ops[j].a; e.cza_layout = S.ops[j].b; ++j; }
      take_phas(&j, end, &e);
      if (j < end && S.ops[j].kind == OP_DIAGT) take_diag(S.ops[j++], &e);
      if (!(j < end && S.ops[j].kind == OP_PERM) || e.pha_count > kEpochMaxPhaseA) {
        // epochs are fused only with their PERM; otherwise the ops stay as they are
        S.phas.resize(e.pha_first);
        if (e.ry_kind == 2 && S.ops[i + (S.ops[i].kind == OP_FUNC ? 1 : 0)].kind == OP_RY) S.rygs.pop_back();
        for (int q = i; q < j; ++q) out.push_back(S.ops[q]);
        i = j;
        continue;
      }
      e.perm_from = S.ops[j].a;
      e.perm_to = S.ops[j].b;
      ++j;
      emit(e);
      i = j;
    }
    *nc = (int)out.size() - *nb;
  };
  for (PassRec& pr : S.passes) {
    int b, c;
    fwd(pr.fop_begin, pr.fop_count, &b, &c);
    pr.fop_begin = b;
    pr.fop_count = c;
    bwd(pr.bop_begin, pr.bop_count, &b, &c);
    pr.bop_begin = b;
    pr.bop_count = c;
  }
  S.ops.swap(out);
}

bool build_schedule(const Circuit& C, const Tuning& T, Schedule* Sp, std::string* msg) {
  Schedule& S = *Sp;
  S = Schedule{};
  const int n = C.n;
  for (const qf_pauli& o : C.obs) S.general_obs = S.general_obs || o.x_mask != 0;
  // default tile: 2^12 amplitudes, 4 register qubits per lane, 256 lanes; the
  // adjoint kernel then holds psi and lambda in 64 VGPRs and keeps 3 waves per SIMD
  const int k = std::min(n, T.k > 0 ? std::min(T.k, kMaxTileQubits) : kDefaultTileQubits);
  const int R = std::min(T.R > 0 ? std::min(T.R, kMaxR) : kDefaultRegQubits, k);
  const int tb = k - R;
  if (tb > kMaxThreadBits) {
    if (msg) *msg = "tile needs more than 256 threads; raise reg_qubits or lower tile_qubits";
    return false;
  }
  const int F = T.fusion > 0 ? T.fusion : (n <= k ? 16 : 8);
  S.n = n;
  S.k = k;
  S.R = R;
  S.thread_bits = tb;
  S.active = 1 << tb;
  // a workgroup is one wave for tiles of up to 64 threads, else exactly the tile's
  // threads: the adjoint pass drops idle lanes' functionals only in 64-thread
  // workgroups, so wider ones must never hold idle lanes
  S.NT = std::max(64, S.active);
  S.tiles_log2 = n - k;
  S.fusion = F;
  S.fill = T.fill == 0 ? R : std::max(0, T.fill);
  std::vector<Unit> units_unused;
  std::vector<std::vector<int>> wire_unused;
  build_runs(C, S, &units_unused, &wire_unused, false);

  // ---- per-wire runs and the diagonal items between them
  // gap g of wire q lies before the wire's run g (gap m_q follows its last run)
  struct Item {
    int kind;        // 0 phase, 1 cz
    int q0, q1;      // qubits (q1 = -1 for a phase)
    int g0, g1;      // gap on q0 / q1
    int ev;          // phase event index (kind 0)
    bool applied = false, released = false, trailing = false;
  };
  std::vector<std::vector<int>> wire_runs(n);
  for (size_t r = 0; r < S.runs.size(); ++r) wire_runs[S.runs[r].q].push_back((int)r);
  std::vector<Item> items;
  std::vector<std::vector<std::vector<int>>> gap_items(n);
  for (int q = 0; q < n; ++q) gap_items[q].resize(wire_runs[q].size() + 1);
  {
    // CZ gates: gap = number of runs of the wire started before the gate
    std::vector<int> started(n, 0);
    std::vector<char> open(n, 0);
    for (const qf_gate& g : C.gates) {
      if (g.kind == QF_CZ) {
        Item it;
        it.kind = 1;
        it.q0 = g.q0;
        it.q1 = g.q1;
        it.g0 = started[g.q0];
        it.g1 = started[g.q1];
        it.ev = -1;
        int id = (int)items.size();
        items.push_back(it);
        gap_items[g.q0][it.g0].push_back(id);
        gap_items[g.q1][it.g1].push_back(id);
        open[g.q0] = open[g.q1] = 0;
      } else if (!open[g.q0]) {
        open[g.q0] = 1;
        started[g.q0]++;
      }
    }
  }
  // phase items: one per gap that borders a run
  for (int q = 0; q < n; ++q) {
    const int m = (int)wire_runs[q].size();
    for (int g = 0; g <= m; ++g) {
      if (m == 0) break;
      EventRec er;
      er.prev_ref = g > 0 ? S.runs[wire_runs[q][g - 1]].coef : INT32_MIN;
      er.next_ref = g < m ? S.runs[wire_runs[q][g]].coef : INT32_MIN;
      er.per_sample = (er.prev_ref != INT32_MIN && er.prev_ref < 0) || (er.next_ref != INT32_MIN && er.next_ref < 0);
      er.pad = 0;
      int ref = er.per_sample ? -1 - (S.n_ev_ps++) : (S.n_ev_shared++);
      Item it;
      it.kind = 0;
      it.q0 = q;
      it.q1 = -1;
      it.g0 = g;
      it.g1 = -1;
      it.ev = (int)S.pev.size();
      S.pev.push_back({q, ref});
      S.events.push_back(er);
      int id = (int)items.size();
      items.push_back(it);
      gap_items[q][g].push_back(id);
    }
  }
  // event table order: shared rows first, then per-sample rows, each by ref
  {
    std::vector<EventRec> ord(S.events.size());
    std::vector<int> sh, ps;
    for (size_t i = 0; i < S.pev.size(); ++i) (S.pev[i].ref >= 0 ? sh : ps).push_back((int)i);
    size_t o = 0;
    for (int i : sh) ord[o++] = S.events[i];
    for (int i : ps) ord[o++] = S.events[i];
    S.events = ord;   // shared rows 0..n_ev_shared-1, per-sample rows after
  }
  for (Item& it : items) {
    const int m0 = (int)wire_runs[it.q0].size();
    it.trailing = it.g0 == m0 && (it.kind == 0 || it.g1 == (int)wire_runs[it.q1].size());
  }

  std::vector<int> runs_done(n, 0);
  int64_t runs_left = (int64_t)S.runs.size();
  std::vector<int> released_list;
  auto try_release = [&](int id) {
    Item& it = items[id];
    if (it.released || it.applied || it.trailing) return;
    if (runs_done[it.q0] < it.g0) return;
    if (it.kind == 1 && runs_done[it.q1] < it.g1) return;
    it.released = true;
    released_list.push_back(id);
  };
  for (size_t i = 0; i < items.size(); ++i) try_release((int)i);
  auto gap_clear = [&](int q) {   // all items before the wire's next run applied
    for (int id : gap_items[q][runs_done[q]])
      if (!items[id].applied) return false;
    return true;
  };
  auto gap_released = [&](int q) {
    for (int id : gap_items[q][runs_done[q]])
      if (!items[id].applied && !items[id].released) return false;
    return true;
  };
  auto has_run = [&](int q) { return runs_done[q] < (int)wire_runs[q].size(); };

  // ---- priority (see the scheduling notes in the header)
  auto earliest_run_wire = [&]() {
    int best = -1, bo = 0;
    for (int q = 0; q < n; ++q) {
      if (!has_run(q)) continue;
      const int gi = S.run_gates[S.runs[wire_runs[q][runs_done[q]]].gate_begin];
      if (best < 0 || gi < bo) { best = q; bo = gi; }
    }
    return best;
  };
  auto by_priority = [&](std::vector<int> qs) {
    const int first = earliest_run_wire();
    std::stable_sort(qs.begin(), qs.end(), [&](int a, int b) {
      if ((a == first) != (b == first)) return a == first;
      bool pa = has_run(a), pb = has_run(b);
      if (pa != pb) return pa;
      if (runs_done[a] != runs_done[b]) return runs_done[a] < runs_done[b];
      return a < b;
    });
    return qs;
  };
  std::vector<int> all(n);
  std::iota(all.begin(), all.end(), 0);
  // core: the qubits at the lowest memory bits, local in consecutive passes so that
  // the passes' loads and stores stay coalesced; a tile that does not hold the
  // whole state keeps at least one position for the qubits it brings in
  const int ncore = n <= k ? std::min(4, k) : std::min(4, k - 1);
  std::vector<int> in_map(n), local;
  std::iota(in_map.begin(), in_map.end(), 0);
  if (n <= k) {
    local = all;
  } else {
    std::vector<int> core, rest;
    for (int q = 0; q < n; ++q) (in_map[q] < ncore ? core : rest).push_back(q);
    rest = by_priority(rest);
    local = core;
    for (int i = 0; (int)local.size() < k; ++i) local.push_back(rest[i]);
  }

  int pass_id = 0;
  const int64_t guard = (int64_t)S.runs.size() * 4 + (int64_t)items.size() + 16;
  while (true) {
    if (pass_id > guard) {
      if (msg) *msg = "scheduler made no progress";
      return false;
    }
    PassRec pr;
    std::memset(&pr, 0, sizeof(pr));
    std::sort(local.begin(), local.end(), [&](int a, int b) { return in_map[a] < in_map[b]; });
    std::vector<int> pos_of(n, -1);
    for (int p = 0; p < k; ++p) pos_of[local[p]] = p;
    {
      std::vector<int> nl;
      for (int q = 0; q < n; ++q)
        if (pos_of[q] < 0) nl.push_back(q);
      std::sort(nl.begin(), nl.end(), [&](int a, int b) { return in_map[a] < in_map[b]; });
      int i = 0;
      for (int q : nl) {
        pr.nl_log[i] = (uint8_t)q;
        pr.nl_in[i] = (uint8_t)in_map[q];
        ++i;
      }
      pr.n_nonlocal = i;
    }
    auto io_layout = [&](const std::vector<int>& map) {
      std::vector<int> by_mem(k);
      std::iota(by_mem.begin(), by_mem.end(), 0);
      std::sort(by_mem.begin(), by_mem.end(), [&](int a, int b) { return map[local[a]] < map[local[b]]; });
      std::vector<int> thr(by_mem.begin(), by_mem.begin() + tb);
      std::vector<int> reg(by_mem.begin() + tb, by_mem.end());
      int id = (int)S.layouts.size();
      S.layouts.push_back(make_layout(reg, thr, local, &map, R));
      return id;
    };
    const int fop_begin = (int)S.ops.size();
    int cur = io_layout(in_map);
    S.ops.push_back({pass_id == 0 ? OP_INIT0 : OP_LOAD, cur, 0, 0, 0, 0, 0, 0});
    std::vector<int> regq(R);
    auto set_regs = [&]() {
      for (int j = 0; j < R; ++j) regq[j] = S.layouts[cur].reg_qubit[j];
    };
    set_regs();
    auto is_reg = [&](int q) { return std::find(regq.begin(), regq.end(), q) != regq.end(); };
    std::vector<int> pass_runs(n, 0);
    int slot = 0;

    // diagonal items whose qubits are all outside the register bits: one factor per thread
    auto apply_free = [&]() {
      std::map<int, uint32_t> groups;
      std::vector<PhaseEv> evs;
      std::vector<int> keep;
      for (int id : released_list) {
        Item& it = items[id];
        if (it.applied) continue;
        if (is_reg(it.q0) || (it.kind == 1 && is_reg(it.q1))) {
          keep.push_back(id);
          continue;
        }
        it.applied = true;
        if (it.kind == 1) {
          int lo = std::min(it.q0, it.q1), hi = std::max(it.q0, it.q1);
          groups[hi - lo] ^= 1u << lo;
        } else {
          evs.push_back(S.pev[it.ev]);
        }
        S.n_diag_thread++;
      }
      released_list = keep;
      std::vector<CzGroup> gs;
      for (auto& kv : groups)
        if (kv.second) gs.push_back({(uint32_t)kv.first, kv.second});
      if (gs.empty() && evs.empty()) return;
      const int cb = (int)S.czg.size(), eb = (int)S.pev.size();
      for (auto& g : gs) S.czg.push_back(g);
      for (auto& e : evs) S.pev.push_back(e);
      S.ops.push_back({OP_DIAGT, cur, cb, (int)gs.size(), eb, (int)evs.size(), 0, 0});
    };
    // diagonal items touching register bits: phases per register bit (PHASEA),
    // CZ signs per amplitude (one CZA for all edges)
    auto apply_amp = [&](const std::vector<int>& ids) {
      std::vector<std::pair<int, int>> edges;
      for (int id : ids) {
        Item& it = items[id];
        if (it.applied) continue;
        it.applied = true;
        S.n_diag_amp++;
        if (it.kind == 1) {
          edges.push_back({it.q0, it.q1});
        } else {
          int j = (int)(std::find(regq.begin(), regq.end(), it.q0) - regq.begin());
          const int eb = (int)S.pev.size();
          S.pev.push_back(S.pev[it.ev]);
          S.ops.push_back({OP_PHASEA, j, eb, 0, 0, 0, 0, 0});
        }
      }
      if (edges.empty()) return;
      CzaRec cr;
      std::memset(&cr, 0, sizeof(cr));
      std::vector<int> rb(n, -1);
      for (int j = 0; j < R; ++j) rb[regq[j]] = j;
      for (auto& e : edges) {
        const int ja = rb[e.first], jbb = rb[e.second];
        if (ja >= 0 && jbb >= 0) {
          for (int jj = 0; jj < (1 << R); ++jj)
            if (((jj >> ja) & 1) && ((jj >> jbb) & 1)) cr.sr ^= 1u << jj;
        } else if (ja >= 0) {
          cr.cmask[ja] ^= 1u << e.second;
        } else {
          cr.cmask[jbb] ^= 1u << e.first;
        }
      }
      S.ops.push_back({OP_CZA, (int)S.cza.size(), cur, 0, 0, 0, 0, 0});
      S.cza.push_back(cr);
      S.n_cz++;
    };

    while (true) {
      // while the pass holds only its LOAD (INIT0), the first exchange is folded
      // into it: the tile is loaded straight into the first epoch's layout
      const bool at_load = S.ops.size() == (size_t)fop_begin + 1;
      if (!at_load) apply_free();
      std::vector<int> cands;
      for (int q : local)
        if (has_run(q) && pass_runs[q] < F && gap_released(q)) cands.push_back(q);
      if (cands.empty()) break;
      // an epoch with fewer than S.fill runs at the end of a pass whose runs
      // are not the circuit's last: leave them to the next pass, where they
      // fill whole epochs (fewer epochs for more passes); a pass that has not
      // done any work yet takes them
      if ((int)cands.size() < S.fill && slot > 0 && runs_left > (int64_t)cands.size()) break;
      // wires whose items are all applied first (no per-amplitude work), then priority
      cands = by_priority(cands);
      std::stable_sort(cands.begin(), cands.end(), [&](int a, int b) { return gap_clear(a) > gap_clear(b); });
      std::vector<int> want(cands.begin(), cands.begin() + std::min<size_t>(R, cands.size()));
      const int n_run_wires = (int)want.size();
      if ((int)want.size() < R) {
        std::vector<int> others;
        for (int q : local)
          if (std::find(want.begin(), want.end(), q) == want.end()) others.push_back(q);
        others = by_priority(others);
        for (int q : others)
          if ((int)want.size() < R) want.push_back(q);
      }
      bool same = true;
      for (int q : want)
        if (!is_reg(q)) same = false;
      if (!same) {
        std::vector<int> reg;
        for (int q : want) reg.push_back(pos_of[q]);
        std::vector<int> free_pos;
        for (int p = 0; p < k; ++p)
          if (std::find(reg.begin(), reg.end(), p) == reg.end()) free_pos.push_back(p);
        std::vector<int> thr = order_thread_positions(free_pos, tb);
        int id = (int)S.layouts.size();
        S.layouts.push_back(make_layout(reg, thr, local, at_load ? &in_map : nullptr, R));
        if (at_load) {
          // the LOAD (INIT0) reads the pass's memory order into this layout: its
          // lanes' reads scatter over the tile's lines, which the caches absorb
          S.ops[fop_begin].a = id;
        } else {
          S.ops.push_back({OP_PERM, cur, id, 0, 0, 0, 0, 0});
          S.n_perm++;
        }
        cur = id;
        set_regs();
        apply_free();
      } else if (at_load) {
        apply_free();
      }
      // items that still block the chosen runs touch register bits: per amplitude
      std::vector<int> run_wires(want.begin(), want.begin() + n_run_wires);
      std::vector<int> blocking;
      for (int q : run_wires)
        for (int id : gap_items[q][runs_done[q]]) blocking.push_back(id);
      apply_amp(blocking);
      for (int j = 0; j < R; ++j) {
        const int q = regq[j];
        if (std::find(run_wires.begin(), run_wires.end(), q) == run_wires.end()) continue;
        const int r = wire_runs[q][runs_done[q]];
        RunRec& rr = S.runs[r];
        rr.pass = pass_id;
        rr.slot = slot++;
        S.ops.push_back({OP_RY, j, rr.coef, r, 0, 0, 0, 0});
        S.n_u2++;
        runs_done[q]++;
        runs_left--;
        pass_runs[q]++;
        for (int id : gap_items[q][runs_done[q]]) try_release(id);
      }
    }
    pr.n_slots = slot;
    const bool last = (runs_left == 0);
    if (last && !S.general_obs) {
      // only trailing diagonal gates remain; they commute with the Z-string
      // observables and change neither E nor the adjoint at the cuts
      S.ops.push_back({OP_EXPECT, cur, 0, 0, 0, 0, 0, 0});
    } else if (last) {
      // observables with X or Y parts: the trailing diagonal gates are applied
      // too, so the stored final state is the circuit's output state, from
      // which a separate kernel forms E and the adjoint seed
      for (size_t id = 0; id < items.size(); ++id)
        if (!items[id].applied && !items[id].released) {
          items[id].released = true;
          released_list.push_back((int)id);
        }
      apply_free();
      apply_amp(released_list);
      released_list.clear();
    }

    std::vector<int> out_map(n);
    std::vector<int> next_local;
    if (n <= k) {
      out_map = in_map;
      next_local = local;
    } else {
      std::vector<int> pr_all = by_priority(all);
      next_local.assign(pr_all.begin(), pr_all.begin() + k);
      auto in_cur = [&](int q) { return pos_of[q] >= 0; };
      auto cnt_overlap = [&]() {
        int c = 0;
        for (int q : next_local) c += in_cur(q);
        return c;
      };
      for (int q : pr_all) {
        if (cnt_overlap() >= ncore) break;
        if (!in_cur(q) || std::find(next_local.begin(), next_local.end(), q) != next_local.end()) continue;
        for (int i = k - 1; i >= 0; --i)
          if (!in_cur(next_local[i])) {
            next_local[i] = q;
            break;
          }
      }
      std::vector<int> shared;
      for (int q : next_local)
        if (in_cur(q)) shared.push_back(q);
      std::vector<int> core;
      for (int r = 0; r < 4 && (int)core.size() < ncore; ++r)
        for (int q : shared)
          if ((pos_of[q] & 3) == r && std::find(core.begin(), core.end(), q) == core.end()) {
            core.push_back(q);
            break;
          }
      for (int q : shared)
        if ((int)core.size() < ncore && std::find(core.begin(), core.end(), q) == core.end()) core.push_back(q);
      int m = 0;
      std::vector<char> placed(n, 0);
      for (int q : core) { out_map[q] = m++; placed[q] = 1; }
      std::vector<int> nl_sorted = next_local;
      std::sort(nl_sorted.begin(), nl_sorted.end());
      for (int q : nl_sorted)
        if (!placed[q]) { out_map[q] = m++; placed[q] = 1; }
      for (int q = 0; q < n; ++q)
        if (!placed[q]) { out_map[q] = m++; placed[q] = 1; }
    }
    for (int i = 0; i < pr.n_nonlocal; ++i) pr.nl_out[i] = (uint8_t)out_map[pr.nl_log[i]];
    // the store layout keeps the last epoch's register and thread positions, with
    // the memory bits of the next pass's order: the tile is stored where it is,
    // without an exchange into memory order (the L2 cache merges the lanes' writes
    // into whole lines; the counted HBM traffic is unchanged)
    int io_out = (int)S.layouts.size();
    {
      LayoutRec L = S.layouts[cur];
      for (int j = 0; j < R; ++j) L.mem_reg[j] = 1u << out_map[L.reg_qubit[j]];
      for (int b = 0; b < tb; ++b) {
        int q = 0;
        while (!((L.log_thr[b] >> q) & 1u)) ++q;
        L.mem_thr[b] = 1u << out_map[q];
      }
      S.layouts.push_back(L);
    }
    cur = io_out;
    set_regs();
    if (!last) apply_free();
    S.ops.push_back({OP_STORE, io_out, 0, 1, 0, 0, 0, 0});
    pr.fop_begin = fop_begin;
    pr.fop_count = (int)S.ops.size() - fop_begin;
    S.passes.push_back(pr);
    ++pass_id;
    if (last) {
      S.final_map.assign(out_map.begin(), out_map.end());
      break;
    }
    in_map = out_map;
    local = next_local;
  }

  // backward programs, mirrored from the forward ones
  const int P = (int)S.passes.size();
  for (int p = 0; p < P; ++p) {
    PassRec& pr = S.passes[p];
    std::vector<Op> f(S.ops.begin() + pr.fop_begin, S.ops.begin() + pr.fop_begin + pr.fop_count);
    std::vector<Op> b;
    const Op st = f.back();
    const Op ld = f.front();
    b.push_back({OP_LOAD, st.a, 0, 1, 0, 0, 0, 0});
    if (p == P - 1 && !S.general_obs) b.push_back({OP_SEED, st.a, 0, 0, 0, 0, 0, 0});
    else b.push_back({OP_LOAD, st.a, 1, 1, 0, 0, 0, 0});   // (general observables: the seed kernel's lambda)
    int i = (int)f.size() - 2;
    while (i >= 1) {
      const Op& o = f[i];
      if (o.kind == OP_RY) {
        // f[j..i]: runs of one register epoch on distinct qubits, nothing in
        // between, so their functionals share one cut
        int j = i;
        uint32_t bits = 1u << f[i].a;
        while (j - 1 >= 1 && f[j - 1].kind == OP_RY && !((bits >> f[j - 1].a) & 1)) {
          --j;
          bits |= 1u << f[j].a;
        }
        int fb = (int)S.funcs.size();
        // one entry per register bit, indexed by the bit; slot -1: no run there
        for (int q = 0; q < R; ++q) S.funcs.push_back({q, -1});
        for (int m = j; m <= i; ++m) S.funcs[fb + f[m].a].slot = S.runs[f[m].c].slot;
        b.push_back({OP_FUNC, R, fb, 0, 0, 0, 0, 0});
        for (int m = i; m >= j; --m) b.push_back(f[m]);
        i = j - 1;
        continue;
      }
      if (o.kind == OP_PERM) b.push_back({OP_PERM, o.b, o.a, 0, 0, 0, 0, 0});
      else if (o.kind == OP_DIAGT || o.kind == OP_CZA || o.kind == OP_PHASEA) b.push_back(o);
      --i;
    }
    if (p > 0) b.push_back({OP_STORE, ld.a, 0, 0, 0, 0, 0, 0});
    pr.bop_begin = (int)S.ops.size();
    pr.bop_count = (int)b.size();
    S.ops.insert(S.ops.end(), b.begin(), b.end());
  }
  group_register_runs(&S);
  fuse_epochs(&S);
  // pass 0 also as a program that loads a given initial state: its input bit
  // order is the logical one, so the state is read as the caller holds it
  for (PassRec& pr : S.passes) pr.fload_begin = -1;
  if (!S.passes.empty() && S.ops[S.passes[0].fop_begin].kind == OP_INIT0) {
    PassRec& p0 = S.passes[0];
    std::vector<Op> f(S.ops.begin() + p0.fop_begin, S.ops.begin() + p0.fop_begin + p0.fop_count);
    f[0] = {OP_LOAD, f[0].a, 0, 0, 0, 0, 0, 0};
    p0.fload_begin = (int)S.ops.size();
    S.ops.insert(S.ops.end(), f.begin(), f.end());
  }
  if (runs_left != 0) {
    if (msg) *msg = "scheduler left runs unapplied";
    return false;
  }
  // runs of each pass in slot order
  S.pass_run_begin.assign(P + 1, 0);
  for (const RunRec& r : S.runs) S.pass_run_begin[r.pass + 1]++;
  for (int p = 0; p < P; ++p) S.pass_run_begin[p + 1] += S.pass_run_begin[p];
  S.pass_runs.assign(S.runs.size(), 0);
  for (size_t r = 0; r < S.runs.size(); ++r)
    S.pass_runs[S.pass_run_begin[S.runs[r].pass] + S.runs[r].slot] = (int)r;
  S.max_slots = 0;
  for (const PassRec& pr : S.passes) S.max_slots = std::max(S.max_slots, pr.n_slots);
  for (const Item& it : items)
    if (!it.applied && !it.trailing) {
      if (msg) *msg = "scheduler left a diagonal gate unapplied";
      return false;
    }
  return true;
}

}  // namespace qf
