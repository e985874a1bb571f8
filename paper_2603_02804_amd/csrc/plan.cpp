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
    if (g.kind < QF_RX || g.kind > QF_CZ) return fail(QF_ERR_INVALID_ARG, "unknown gate kind" + at);
    if (g.q0 < 0 || g.q0 >= n) return fail(QF_ERR_INVALID_ARG, "qubit out of range" + at);
    if (g.kind == QF_CZ) {
      if (g.q1 < 0 || g.q1 >= n) return fail(QF_ERR_INVALID_ARG, "CZ partner out of range" + at);
      if (g.q1 == g.q0) return fail(QF_ERR_INVALID_ARG, "CZ on a single qubit" + at);
      if (g.theta_idx != -1 || g.input_idx != -1)
        return fail(QF_ERR_INVALID_ARG, "CZ carries no angle" + at);
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
    if (d->obs[k].x_mask != 0)
      return fail(QF_ERR_UNSUPPORTED, "only Z-string observables (x_mask == 0) are implemented");
  }
  return QF_OK;
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
  for (int j = 0; j < kMaxR; ++j) L.reg_qubit[j] = (j < R) ? local[reg_pos[j]] : -1;
  for (int jj = 0; jj < (1 << R); ++jj) {
    uint32_t lds = 0, lg = 0, mem = 0;
    for (int j = 0; j < R; ++j)
      if ((jj >> j) & 1) {
        lds ^= lds_swizzle(1u << reg_pos[j]);
        lg |= 1u << local[reg_pos[j]];
        if (map) mem |= 1u << (*map)[local[reg_pos[j]]];
      }
    L.lds_reg[jj] = lds;
    L.log_reg[jj] = lg;
    L.mem_reg[jj] = mem;
  }
  for (size_t b = 0; b < thr_pos.size(); ++b) {
    L.lds_thr[b] = lds_swizzle(1u << thr_pos[b]);
    L.log_thr[b] = 1u << local[thr_pos[b]];
    L.mem_thr[b] = map ? (1u << (*map)[local[thr_pos[b]]]) : 0u;
  }
  return L;
}

// Orders thread positions so that lanes 0..3 take distinct residues mod 4 of
// their tile positions (conflict-free 64-bit LDS accesses with the swizzle).
std::vector<int> order_thread_positions(std::vector<int> free_pos, int tb) {
  std::vector<int> out;
  for (int r = 0; r < 4 && (int)out.size() < std::min(tb, 4); ++r) {
    for (size_t i = 0; i < free_pos.size(); ++i)
      if ((free_pos[i] & 3) == r) {
        out.push_back(free_pos[i]);
        free_pos.erase(free_pos.begin() + i);
        break;
      }
  }
  for (int p : free_pos) out.push_back(p);
  out.resize(tb);
  return out;
}

}  // namespace

void build_gate_runs(const Circuit& c, Schedule* s) {
  build_runs(c, *s, nullptr, nullptr, true);
}

bool build_schedule(const Circuit& C, const Tuning& T, Schedule* Sp, std::string* msg) {
  Schedule& S = *Sp;
  S = Schedule{};
  Builder B(C, S);
  const int n = C.n;
  B.n = n;
  int kmax = T.k > 0 ? std::min(T.k, kMaxTileQubits) : kMaxTileQubits;
  B.k = std::min(n, kmax);
  B.R = std::min(T.R > 0 ? std::min(T.R, kMaxR) : kMaxR, B.k);
  B.tb = B.k - B.R;
  if (B.tb > kMaxThreadBits) {
    if (msg) *msg = "tile needs more than 256 threads; raise reg_qubits or lower tile_qubits";
    return false;
  }
  B.F = T.fusion > 0 ? T.fusion : (n <= B.k ? 16 : 8);
  S.n = n;
  S.k = B.k;
  S.R = B.R;
  S.thread_bits = B.tb;
  S.active = 1 << B.tb;
  S.NT = std::max(64, S.active);
  S.tiles_log2 = n - B.k;
  S.fusion = B.F;
  build_runs(C, S, &B.units, &B.wire, false);
  B.ptr.assign(n, 0);
  B.depth.assign(n, 0);
  B.remaining = (int64_t)B.units.size();
  const int k = B.k, R = B.R, tb = B.tb, F = B.F;
  const int ncore = std::min(4, k);

  std::vector<int> in_map(n), local;
  std::iota(in_map.begin(), in_map.end(), 0);

  // priority: the wire of the earliest pending run in circuit order (which is
  // always ready once ready CZs are applied, so every pass makes progress), then
  // wires with pending units, least advanced first
  auto earliest_run_wire = [&]() {
    int best = -1, bo = 0;
    for (int q = 0; q < n; ++q) {
      int u = B.front(q);
      if (u >= 0 && B.units[u].kind == 0 && (best < 0 || B.units[u].order < bo)) {
        best = q;
        bo = B.units[u].order;
      }
    }
    return best;
  };
  auto by_priority = [&](std::vector<int> qs) {
    const int first = earliest_run_wire();
    std::stable_sort(qs.begin(), qs.end(), [&](int a, int b) {
      if ((a == first) != (b == first)) return a == first;
      bool pa = B.front(a) >= 0, pb = B.front(b) >= 0;
      if (pa != pb) return pa;
      if (B.depth[a] != B.depth[b]) return B.depth[a] < B.depth[b];
      return a < b;
    });
    return qs;
  };
  std::vector<int> all(n);
  std::iota(all.begin(), all.end(), 0);

  // initial local set: memory core + least advanced
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
  const int64_t guard = (int64_t)B.units.size() * 4 + 16;
  while (true) {
    if (pass_id > guard) {
      if (msg) *msg = "scheduler made no progress";
      return false;
    }
    PassRec pr;
    std::memset(&pr, 0, sizeof(pr));
    // tile positions: in-memory order of the local qubits (core first)
    std::sort(local.begin(), local.end(), [&](int a, int b) { return in_map[a] < in_map[b]; });
    std::vector<int> pos_of(n, -1);
    for (int p = 0; p < k; ++p) pos_of[local[p]] = p;
    {
      int i = 0;
      std::vector<int> nl;
      for (int q = 0; q < n; ++q)
        if (pos_of[q] < 0) nl.push_back(q);
      std::sort(nl.begin(), nl.end(), [&](int a, int b) { return in_map[a] < in_map[b]; });
      for (int q : nl) {
        pr.nl_log[i] = (uint8_t)q;
        pr.nl_in[i] = (uint8_t)in_map[q];
        ++i;
      }
      pr.n_nonlocal = i;
    }
    // load layout: lanes on the lowest memory bits
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
    S.ops.push_back({pass_id == 0 ? OP_INIT0 : OP_LOAD, cur, 0, 0});
    std::vector<int> regq(R, -1);   // qubit in each register bit of `cur` (unknown for io)
    for (int j = 0; j < R; ++j) regq[j] = S.layouts[cur].reg_qubit[j];
    std::vector<int> pass_runs(n, 0);
    int slot = 0;

    auto apply_ready_czs = [&]() {
      std::map<int, uint32_t> groups;
      bool found = true;
      while (found) {
        found = false;
        for (int q = 0; q < n; ++q) {
          int u = B.front(q);
          if (u < 0 || B.units[u].kind != 1 || B.units[u].a != q || !B.ready(u)) continue;
          int lo = std::min(B.units[u].a, B.units[u].b), hi = std::max(B.units[u].a, B.units[u].b);
          groups[hi - lo] ^= 1u << lo;   // CZ twice on the same pair cancels
          B.finish(u);
          found = true;
        }
      }
      std::vector<CzGroup> gs;
      for (auto& kv : groups)
        if (kv.second) gs.push_back({(uint32_t)kv.first, kv.second});
      if (!gs.empty()) {
        S.ops.push_back({OP_CZ, cur, (int32_t)S.czg.size(), (int32_t)gs.size()});
        for (auto& g : gs) S.czg.push_back(g);
        S.n_cz++;
      }
    };
    auto runnable = [&](int q) {
      int u = B.front(q);
      return u >= 0 && B.units[u].kind == 0 && pass_runs[q] < F;
    };

    while (true) {
      apply_ready_czs();
      std::vector<int> cands;
      for (int q : local)
        if (runnable(q)) cands.push_back(q);
      if (cands.empty()) break;
      cands = by_priority(cands);
      // register set: ready runs first, then local wires whose next run waits on a CZ
      std::vector<int> want(cands.begin(), cands.begin() + std::min<size_t>(R, cands.size()));
      if ((int)want.size() < R) {
        std::vector<int> others;
        for (int q : local)
          if (std::find(want.begin(), want.end(), q) == want.end() && B.front(q) >= 0 && pass_runs[q] < F)
            others.push_back(q);
        others = by_priority(others);
        for (int q : others)
          if ((int)want.size() < R) want.push_back(q);
      }
      bool same = true;
      for (int q : want)
        if (std::find(regq.begin(), regq.end(), q) == regq.end()) same = false;
      if (!same) {
        // fill the register bits, then order the thread positions
        std::vector<int> reg;
        for (int q : want) reg.push_back(pos_of[q]);
        std::vector<int> free_pos;
        for (int p = 0; p < k; ++p)
          if (std::find(reg.begin(), reg.end(), p) == reg.end()) free_pos.push_back(p);
        // fillers: prefer residues mod 4 with the most free positions left
        while ((int)reg.size() < R) {
          int cnt[4] = {0, 0, 0, 0};
          for (int p : free_pos) cnt[p & 3]++;
          int best = 0;
          for (int i = 1; i < (int)free_pos.size(); ++i)
            if (cnt[free_pos[i] & 3] > cnt[free_pos[best] & 3]) best = i;
          reg.push_back(free_pos[best]);
          free_pos.erase(free_pos.begin() + best);
        }
        std::vector<int> thr = order_thread_positions(free_pos, tb);
        int id = (int)S.layouts.size();
        S.layouts.push_back(make_layout(reg, thr, local, nullptr, R));
        S.ops.push_back({OP_PERM, cur, id, 0});
        S.n_perm++;
        cur = id;
        for (int j = 0; j < R; ++j) regq[j] = S.layouts[cur].reg_qubit[j];
      }
      bool progress = true;
      while (progress) {
        progress = false;
        for (int j = 0; j < R; ++j) {
          int q = regq[j];
          if (q < 0 || !runnable(q)) continue;
          int u = B.front(q);
          int r = B.units[u].run;
          RunRec& rr = S.runs[r];
          rr.pass = pass_id;
          rr.slot = slot++;
          S.ops.push_back({OP_U2, j, rr.coef, r});
          S.n_u2++;
          B.finish(u);
          pass_runs[q]++;
          progress = true;
        }
        if (progress) apply_ready_czs();
      }
    }
    pr.n_slots = slot;
    const bool last = (B.remaining == 0);
    if (last) S.ops.push_back({OP_EXPECT, cur, 0, 0});

    // next local set and the memory map after this pass
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
      // keep at least `ncore` qubits of this tile so both passes stream >=128-byte rows
      for (int q : pr_all) {
        if (cnt_overlap() >= ncore) break;
        if (!in_cur(q) || std::find(next_local.begin(), next_local.end(), q) != next_local.end()) continue;
        for (int i = k - 1; i >= 0; --i)
          if (!in_cur(next_local[i])) {
            next_local[i] = q;
            break;
          }
      }
      // memory core: shared qubits, distinct tile-position residues if possible
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
    int io_out = io_layout(out_map);
    if (io_out != cur) S.ops.push_back({OP_PERM, cur, io_out, 0});
    S.ops.push_back({OP_STORE, io_out, 0, 1});
    pr.fop_begin = fop_begin;
    pr.fop_count = (int)S.ops.size() - fop_begin;
    S.passes.push_back(pr);
    ++pass_id;
    if (last) break;
    in_map = out_map;
    local = next_local;
  }

  // backward programs, mirrored from the forward ones
  const int P = (int)S.passes.size();
  for (int p = 0; p < P; ++p) {
    PassRec& pr = S.passes[p];
    std::vector<Op> f(S.ops.begin() + pr.fop_begin, S.ops.begin() + pr.fop_begin + pr.fop_count);
    std::vector<Op> b;
    const Op& st = f.back();        // STORE with the output layout
    const Op& ld = f.front();       // LOAD / INIT0 with the input layout
    b.push_back({OP_LOAD, st.a, 0, 1});
    if (p == P - 1) b.push_back({OP_SEED, st.a, 0, 0});
    else b.push_back({OP_LOAD, st.a, 1, 1});
    int i = (int)f.size() - 2;
    while (i >= 1) {
      const Op& o = f[i];
      if (o.kind == OP_U2) {
        // f[j..i]: consecutive runs on distinct register bits (distinct qubits,
        // nothing in between), so their functionals share one cut
        int j = i;
        uint32_t bits = 1u << f[i].a;
        while (j - 1 >= 1 && f[j - 1].kind == OP_U2 && !((bits >> f[j - 1].a) & 1)) {
          --j;
          bits |= 1u << f[j].a;
        }
        int fb = (int)S.funcs.size();
        for (int m = j; m <= i; ++m) S.funcs.push_back({f[m].a, S.runs[f[m].c].slot});
        b.push_back({OP_FUNC, i - j + 1, fb, 0});
        for (int m = i; m >= j; --m) b.push_back({OP_U2ADJ, f[m].a, f[m].b, f[m].c});
        i = j - 1;
        continue;
      }
      if (o.kind == OP_PERM) b.push_back({OP_PERM, o.b, o.a, 0});
      else if (o.kind == OP_CZ) b.push_back(o);
      // OP_EXPECT: nothing to undo
      --i;
    }
    if (p > 0) b.push_back({OP_STORE, ld.a, 0, 0});
    pr.bop_begin = (int)S.ops.size();
    pr.bop_count = (int)b.size();
    S.ops.insert(S.ops.end(), b.begin(), b.end());
  }
  // sanity: every unit applied exactly once
  if (B.remaining != 0) {
    if (msg) *msg = "scheduler left gates unapplied";
    return false;
  }
  for (const RunRec& r : S.runs)
    if (r.pass < 0) {
      if (msg) *msg = "run without a pass";
      return false;
    }
  return true;
}

}  // namespace qf
