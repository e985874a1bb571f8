// batch.hpp -- mixed batches of circuits (host side).
//
// Every circuit of a mixed batch keeps its own plan.  Its forward or backward
// call is first recorded as the sequence of launches the single-plan driver
// would issue (driver.hpp), with workspace addresses kept as offsets into one
// batch workspace and caller buffers left to a per-circuit pointer table.  The
// sequences are then merged step by step: step s launches, for every compiled
// pass kernel variant and once for the small kernels, ONE kernel that runs the
// s-th launch of every circuit whose s-th launch is of that kind.  Launches of
// one circuit stay in order (they are consecutive steps on one stream); launches
// of different circuits are independent.  The merged launch count is about the
// longest circuit's sequence instead of the sum over circuits, and the small
// circuits fill the device together instead of one at a time.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "small_args.hpp"

namespace qf {

// Default end-of-pass epoch threshold of the plans of a mixed batch (tuning
// epoch_fill 0): an end-of-pass epoch of fewer than 2 runs waits for the next
// pass.  Merged launches advance every circuit one pass per step, so extra passes
// cost steps; with the heaviest group split over two streams the fewer epochs
// gain more (mixed256: 1.1% faster than no deferral, which is faster with one
// stream).
constexpr int kBatchEpochFill = 2;

// The heaviest tile-shape group of a mixed batch is merged as this many parts of
// equal weight that run on streams of their own (see merge_grouped).
constexpr int kHeaviestGroupParts = 2;

// Default fusion depth of the plans of a mixed batch whose circuits exceed one
// tile (tuning fusion_depth 0): deeper than a single plan's, since every pass
// costs a merged step (smaller circuits keep the single-plan default).
constexpr int kBatchFusionDepth = 12;

// The tuning of one circuit's plan in a mixed batch: the batch's tuning, whose
// zero fields take the batch defaults above.
inline qf_tuning batch_plan_tuning(const qf_tuning& bt, int n_qubits) {
  qf_tuning t = bt;
  if (t.epoch_fill == 0) t.epoch_fill = kBatchEpochFill;
  const int k = t.tile_qubits > 0 ? t.tile_qubits : kDefaultTileQubits;
  if (t.fusion_depth == 0 && n_qubits > k) t.fusion_depth = kBatchFusionDepth;
  return t;
}

// Compiled pass kernel variants: register qubits R in 1..5, NT in {64,128,256},
// forward or backward.
constexpr int kPassClasses = 30;

inline int pass_class(int R, int NT, bool bwd) {
  const int nt = NT == 64 ? 0 : NT == 128 ? 1 : NT == 256 ? 2 : -1;
  if (nt < 0 || R < 1 || R > 5) return -1;
  return ((R - 1) * 3 + nt) * 2 + (bwd ? 1 : 0);
}
inline int class_R(int cls) { return cls / 6 + 1; }
inline int class_NT(int cls) { return 64 << ((cls / 2) % 3); }
inline bool class_bwd(int cls) { return (cls & 1) != 0; }

struct JobRec {
  int cls;            // pass class, or -1 for a small-kernel job
  int idx;            // index into the circuit's pass or small jobs
};

// One circuit's recorded launch sequence.
struct CircProgram {
  std::vector<JobRec> recs;
  std::vector<PassJob> pj;
  std::vector<PassLaunch> pl;       // the driver's view of each pass job (host checks)
  std::vector<uint32_t> pblocks, pshmem;
  std::vector<uint32_t> pcost;      // work per workgroup of each pass job (its runs, plus the tile load and store)
  std::vector<SmallJob> sj;
  std::vector<uint32_t> sblocks, sshmem;
};

// Exec backend of driver.hpp that records instead of launching.  `ws` given to
// the driver is a fake base equal to the circuit's offset in the batch
// workspace, so every workspace address it forms is that offset.
struct RecordExec {
  const PlanCore& c;
  const PlanPtrs& d;
  int circ;
  CircProgram& out;
  CoefPtrs cp;
  RecordExec(const PlanCore& pc, const PlanPtrs& dp, int ci, CircProgram& o) : c(pc), d(dp), circ(ci), out(o) {}
  qf_status status() const { return QF_OK; }

  void small(const SmallJob& j, long long blocks, size_t shmem) {
    out.recs.push_back({-1, (int)out.sj.size()});
    out.sj.push_back(j);
    out.sblocks.push_back((uint32_t)blocks);
    out.sshmem.push_back((uint32_t)shmem);
  }
  static SmallJob job(int kind, int circ) {
    SmallJob j;
    std::memset(&j, 0, sizeof(j));
    j.kind = kind;
    j.circ = circ;
    return j;
  }
  void coef(const float*, const float*, char* ws) {
    cp = coef_ptrs(c, ws);
    SmallJob j = job(SJ_COEF, circ);
    j.u.coef = make_coef_args(c, d, nullptr, nullptr, cp);
    const long long n = coef_items(j.u.coef);
    if (n > 0) small(j, blocks_for(n), 0);
    SmallJob e = job(SJ_EVENT, circ);
    e.u.ev = make_event_args(c, d, cp);
    const long long ne = event_items(e.u.ev);
    if (ne > 0) small(e, blocks_for(ne), 0);
  }
  void pass(const PassLaunch& L) {
    PassJob j;
    std::memset(&j, 0, sizeof(j));
    j.A = make_pass_args(c, d, cp, L);
    j.A.dE = nullptr;
    j.circ = circ;
    j.pass = L.pass;
    out.recs.push_back({pass_class(c.S.R, c.S.NT, L.bwd), (int)out.pj.size()});
    out.pj.push_back(j);
    out.pl.push_back(L);
    out.pblocks.push_back(pass_blocks(c, L.nb));
    out.pshmem.push_back((uint32_t)pass_shmem(c, L.bwd));
    const int p = L.pass;
    const int runs = p + 1 < (int)c.S.pass_run_begin.size() ? c.S.pass_run_begin[p + 1] - c.S.pass_run_begin[p] : 0;
    out.pcost.push_back((uint32_t)(runs + 8));
  }
  // circuits with X / Y observables are rejected at batch creation
  void pauli_expect(const float*, int64_t, int, float*) { failed = true; }
  void pauli_reduce_E(int, int, const float*, float*) { failed = true; }
  void pauli_seed(const float*, int64_t, float*, int64_t, int, int, const float*) { failed = true; }
  bool failed = false;
  void reduce_E(int nb, int sample0, const float* partE, float*) {
    SmallJob j = job(SJ_REDUCE_E, circ);
    j.u.re = make_reduce_E_args<float>(c, nb, sample0, c.tiles * c.waves, partE, nullptr);
    small(j, blocks_for((long long)nb * c.C.K), 0);
  }
  void assemble(int seg, int nb, int sample0, const float*, const float*, const float* partF, float* Gr) {
    SmallJob j = job(SJ_ASSEMBLE, circ);
    j.u.as = make_assemble_args(c, d, seg, nb, sample0, nullptr, nullptr, partF, Gr);
    if (j.u.as.np == 0 || nb == 0) return;
    small(j, (long long)nb * j.u.as.np, assemble_shmem(c));
  }
  void reduce_grads(int nb, int sample0, const float* Gr, float*, float*, bool accumulate) {
    SmallJob j = job(SJ_REDUCE_G, circ);
    j.u.rg = make_reduce_grads_args<float>(c, d, nb, sample0, Gr, nullptr, nullptr, accumulate);
    if (j.u.rg.P > 0 || j.u.rg.dx_items() > 0) small(j, reduce_grads_blocks(j.u.rg), reduce_grads_shmem());
  }
};

struct MergedLaunch {
  int cls;            // pass class, or -1: small kernels
  int32_t job0;       // first job in the pass or small job table
  int32_t n_jobs;
  uint32_t blocks;
  uint32_t shmem;
  int group = 0;      // circuits of one tile shape: groups run on streams of their own
};

struct Program {
  std::vector<MergedLaunch> launches;
  std::vector<PassJob> pjobs;
  std::vector<PassLaunch> plaunch;  // host view of each pass job
  std::vector<int32_t> pstart;      // first block of each job within its launch
  std::vector<SmallJob> sjobs;
  std::vector<int32_t> sstart;
  int steps = 0;
  int64_t jobs = 0;                 // launches of the circuits one by one
  int groups = 1;                   // independent launch sequences (one per tile shape)
};

// Job order of one merged pass launch.  Each XCD runs one contiguous eighth of
// the blocks, so the order spreads the work evenly over them: jobs are taken
// costliest first, each time the one that keeps the running sum of work closest
// to (average work per block) x (running sum of blocks).  Every XCD then ends its
// range at about the same time, while each job stays contiguous (its circuit's
// tables on one XCD).
inline void balance_pass_jobs(const std::vector<CircProgram>& cps, std::vector<std::pair<int, int>>* jobs) {
  std::vector<std::pair<int, int>> rem = *jobs;
  auto blocks = [&](const std::pair<int, int>& j) { return (double)cps[j.first].pblocks[j.second]; };
  auto cost = [&](const std::pair<int, int>& j) { return (double)cps[j.first].pcost[j.second]; };
  std::stable_sort(rem.begin(), rem.end(), [&](const std::pair<int, int>& a, const std::pair<int, int>& b) {
    return cost(a) > cost(b);
  });
  double tb = 0, tw = 0;
  for (auto& j : rem) { tb += blocks(j); tw += blocks(j) * cost(j); }
  const double avg = tb > 0 ? tw / tb : 0;
  jobs->clear();
  double cb = 0, cw = 0;
  while (!rem.empty()) {
    size_t best = 0;
    double bd = -1;
    for (size_t i = 0; i < rem.size(); ++i) {
      const double d = std::fabs(cw + blocks(rem[i]) * cost(rem[i]) - avg * (cb + blocks(rem[i])));
      if (bd < 0 || d < bd) { bd = d; best = i; }
    }
    cb += blocks(rem[best]);
    cw += blocks(rem[best]) * cost(rem[best]);
    jobs->push_back(rem[best]);
    rem.erase(rem.begin() + best);
  }
}

// Merges the circuits' sequences; within a small-kernel launch, jobs follow
// `order`; within a pass launch, `balance_pass_jobs` orders them.
inline bool merge_programs(const std::vector<CircProgram>& cps, const std::vector<int>& order, Program* P,
                           std::string* msg) {
  *P = Program{};
  size_t steps = 0;
  for (const CircProgram& cp : cps) steps = std::max(steps, cp.recs.size());
  P->steps = (int)steps;
  std::vector<std::vector<std::pair<int, int>>> by(kPassClasses + 1);
  for (size_t s = 0; s < steps; ++s) {
    for (auto& v : by) v.clear();
    for (int c : order) {
      const CircProgram& cp = cps[c];
      if (s >= cp.recs.size()) continue;
      const JobRec& r = cp.recs[s];
      if (r.cls < -1 || r.cls >= kPassClasses) {
        if (msg) *msg = "no pass kernel variant for a circuit's tile shape";
        return false;
      }
      by[r.cls + 1].push_back({c, r.idx});
    }
    for (int k = 0; k <= kPassClasses; ++k) {
      if (by[k].empty()) continue;
      MergedLaunch L;
      L.cls = k - 1;
      L.blocks = 0;
      L.shmem = 0;
      uint64_t blocks = 0;
      if (L.cls >= 0) {
        balance_pass_jobs(cps, &by[k]);
        L.job0 = (int32_t)P->pjobs.size();
        for (auto& cj : by[k]) {
          const CircProgram& cp = cps[cj.first];
          P->pstart.push_back((int32_t)blocks);
          P->pjobs.push_back(cp.pj[cj.second]);
          P->plaunch.push_back(cp.pl[cj.second]);
          blocks += cp.pblocks[cj.second];
          L.shmem = std::max(L.shmem, cp.pshmem[cj.second]);
        }
      } else {
        L.job0 = (int32_t)P->sjobs.size();
        for (auto& cj : by[k]) {
          const CircProgram& cp = cps[cj.first];
          P->sstart.push_back((int32_t)blocks);
          P->sjobs.push_back(cp.sj[cj.second]);
          blocks += cp.sblocks[cj.second];
          L.shmem = std::max(L.shmem, cp.sshmem[cj.second]);
        }
      }
      if (blocks >= (uint64_t(1) << 31)) {
        if (msg) *msg = "merged launch exceeds the grid size limit";
        return false;
      }
      L.n_jobs = (int32_t)by[k].size();
      L.blocks = (uint32_t)blocks;
      P->jobs += L.n_jobs;
      P->launches.push_back(L);
    }
  }
  return true;
}

// Circuits grouped by tile shape (the pass kernel variant their plan uses), each
// group merged on its own: the groups share no launch, so the caller can run
// them concurrently.  The heaviest group is split in parts of equal weight.
// Groups are ordered by work, heaviest first; `order` keeps its order inside
// each group.  The job tables of all groups are concatenated.
inline bool merge_grouped(const std::vector<CircProgram>& cps, const std::vector<const PlanCore*>& cores,
                          const std::vector<int>& order, Program* P, std::string* msg) {
  std::vector<int> keys;
  std::vector<std::vector<int>> members;
  std::vector<double> weight;
  for (int c : order) {
    const int key = pass_class(cores[c]->S.R, cores[c]->S.NT, false);
    size_t g = 0;
    while (g < keys.size() && keys[g] != key) ++g;
    if (g == keys.size()) {
      keys.push_back(key);
      members.emplace_back();
      weight.push_back(0.0);
    }
    members[g].push_back(c);
    weight[g] += (double)cores[c]->amps * cores[c]->P * cores[c]->B;
  }
  // the heaviest group in parts of equal weight on streams of their own: each
  // part's launches fill the workgroup slots that the others' launch tails leave
  if (kHeaviestGroupParts > 1 && !members.empty()) {
    size_t h = 0;
    for (size_t g = 1; g < members.size(); ++g)
      if (weight[g] > weight[h]) h = g;
    const int parts = (int)std::min<size_t>(kHeaviestGroupParts, members[h].size());
    if (parts > 1) {
      std::vector<std::vector<int>> pm(parts);
      std::vector<double> pw(parts, 0.0);
      for (int c : members[h]) {   // heaviest first (`order`), each to the lightest part
        int m = 0;
        for (int i = 1; i < parts; ++i)
          if (pw[i] < pw[m]) m = i;
        pm[m].push_back(c);
        pw[m] += (double)cores[c]->amps * cores[c]->P * cores[c]->B;
      }
      members[h] = pm[0];
      weight[h] = pw[0];
      for (int i = 1; i < parts; ++i) {
        keys.push_back(keys[h]);
        members.push_back(pm[i]);
        weight.push_back(pw[i]);
      }
    }
  }
  std::vector<size_t> gorder(keys.size());
  for (size_t g = 0; g < gorder.size(); ++g) gorder[g] = g;
  std::stable_sort(gorder.begin(), gorder.end(), [&](size_t a, size_t b) { return weight[a] > weight[b]; });
  *P = Program{};
  P->groups = (int)keys.size();
  for (size_t gi = 0; gi < gorder.size(); ++gi) {
    Program G;
    if (!merge_programs(cps, members[gorder[gi]], &G, msg)) return false;
    const int32_t pj0 = (int32_t)P->pjobs.size(), sj0 = (int32_t)P->sjobs.size();
    for (MergedLaunch L : G.launches) {
      L.job0 += L.cls >= 0 ? pj0 : sj0;
      L.group = (int)gi;
      P->launches.push_back(L);
    }
    P->pjobs.insert(P->pjobs.end(), G.pjobs.begin(), G.pjobs.end());
    P->plaunch.insert(P->plaunch.end(), G.plaunch.begin(), G.plaunch.end());
    P->pstart.insert(P->pstart.end(), G.pstart.begin(), G.pstart.end());
    P->sjobs.insert(P->sjobs.end(), G.sjobs.begin(), G.sjobs.end());
    P->sstart.insert(P->sstart.end(), G.sstart.begin(), G.sstart.end());
    P->steps = std::max(P->steps, G.steps);
    P->jobs += G.jobs;
  }
  return true;
}

// Circuit order of the merged small-kernel launches (and the starting order of
// the pass launches' balancing): heavier circuits (amplitudes x passes x
// samples) first, so that their workgroups are dispatched first.
inline std::vector<int> batch_order(const std::vector<const PlanCore*>& cores) {
  std::vector<int> order(cores.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double wa = (double)cores[a]->amps * cores[a]->P * cores[a]->B;
    const double wb = (double)cores[b]->amps * cores[b]->P * cores[b]->B;
    return wa > wb;
  });
  return order;
}

// Workspace layout of a batch: circuit regions in order, 256-byte aligned, the
// first 256 bytes unused so that no region starts at offset 0.
inline uint64_t batch_layout(const std::vector<const PlanCore*>& cores, std::vector<uint64_t>* off) {
  uint64_t o = 256;
  off->clear();
  for (const PlanCore* c : cores) {
    off->push_back(o);
    o = align_up(o + c->ws_bytes);
  }
  return o;
}

// ---------------------------------------------------------------- bounds checks
// Every workspace address of every job, with the extent the kernels reach from
// it, must lie inside its circuit's workspace region [lo, hi).
struct Region {
  uint64_t lo, hi;
};

inline bool in_region(const void* p, uint64_t bytes, const Region& r) {
  if (!p) return true;
  const uint64_t a = (uint64_t)(uintptr_t)p;
  return a >= r.lo && a + bytes <= r.hi;
}

inline bool check_pass_job(const PassJob& j, const PlanCore& c, uint32_t blocks, const Region& r) {
  const KArgs& A = j.A;
  const Schedule& S = c.S;
  const uint64_t nb = blocks >> S.tiles_log2;
  if (nb == 0 || ((uint64_t)nb << S.tiles_log2) != blocks) return false;
  const uint64_t amps = uint64_t(1) << c.C.n;
  auto state_ext = [&](long long stride, int bf16) { return ((nb - 1) * (uint64_t)stride + amps) * (bf16 ? 4 : 8); };
  if (j.pass < 0 || j.pass >= (int)S.passes.size()) return false;
  const uint64_t ns = (uint64_t)S.passes[j.pass].n_slots;
  bool ok = true;
  ok &= in_region(A.src0, state_ext(A.s0, A.src0_bf16), r);
  ok &= in_region(A.src1, state_ext(A.s1, 0), r);
  ok &= in_region(A.dst, state_ext(A.sd, 0), r);
  ok &= in_region(A.dst2, state_ext(A.sd2, 1), r);
  ok &= in_region(A.dpsi, state_ext(A.sdp, 0), r);
  ok &= in_region(A.partF, nb * c.tiles * 3 * ns * 4, r);
  ok &= in_region(A.partE, nb * c.tiles * (uint64_t)c.waves * c.C.K * 4, r);
  ok &= in_region(A.coef_sh, 32ull * std::max(1, S.n_coef_shared), r);
  ok &= in_region(A.coef_ps, 32ull * std::max<int64_t>(1, (int64_t)c.B * S.n_coef_ps), r);
  ok &= in_region(A.ev_sh, 8ull * std::max(1, S.n_ev_shared), r);
  ok &= in_region(A.ev_ps, 8ull * std::max<int64_t>(1, (int64_t)c.B * S.n_ev_ps), r);
  ok &= (uint64_t)A.sample0 + nb <= (uint64_t)c.B;
  return ok;
}

inline bool check_small_job(const SmallJob& j, const PlanCore& c, const Region& r) {
  const Schedule& S = c.S;
  const uint64_t coef_sh = 32ull * std::max(1, S.n_coef_shared);
  const uint64_t coef_ps = 32ull * std::max<int64_t>(1, (int64_t)c.B * S.n_coef_ps);
  switch (j.kind) {
    case SJ_COEF:
      return in_region(j.u.coef.csh, coef_sh, r) && in_region(j.u.coef.cps, coef_ps, r);
    case SJ_EVENT:
      return in_region(j.u.ev.csh, coef_sh, r) && in_region(j.u.ev.cps, coef_ps, r) &&
             in_region(j.u.ev.esh, 8ull * std::max(1, S.n_ev_shared), r) &&
             in_region(j.u.ev.eps, 8ull * std::max<int64_t>(1, (int64_t)c.B * S.n_ev_ps), r);
    case SJ_REDUCE_E:
      return in_region(j.u.re.partE, (uint64_t)j.u.re.nb * j.u.re.parts * c.C.K * 4, r) &&
             (uint64_t)j.u.re.sample0 + j.u.re.nb <= (uint64_t)c.B;
    case SJ_ASSEMBLE:
      return in_region(j.u.as.partF, (uint64_t)j.u.as.nb * c.partF_seg_floats * 4, r) &&
             in_region(j.u.as.Gr, (uint64_t)j.u.as.nb * c.n_angle * 4, r) &&
             (uint64_t)j.u.as.sample0 + j.u.as.nb <= (uint64_t)c.B;
    case SJ_REDUCE_G:
      return in_region(j.u.rg.Gr, (uint64_t)j.u.rg.nb * c.n_angle * 4, r) &&
             (uint64_t)j.u.rg.sample0 + j.u.rg.nb <= (uint64_t)c.B;
    default:
      return false;
  }
}

inline bool check_program(const std::vector<CircProgram>& cps, const std::vector<const PlanCore*>& cores,
                          const std::vector<Region>& regions, std::string* msg) {
  for (size_t ci = 0; ci < cps.size(); ++ci) {
    const CircProgram& cp = cps[ci];
    for (size_t i = 0; i < cp.pj.size(); ++i)
      if (cp.pj[i].circ != (int)ci || !check_pass_job(cp.pj[i], *cores[ci], cp.pblocks[i], regions[ci])) {
        if (msg) *msg = "pass job " + std::to_string(i) + " of circuit " + std::to_string(ci) +
                        " reaches outside its workspace region";
        return false;
      }
    for (size_t i = 0; i < cp.sj.size(); ++i)
      if (cp.sj[i].circ != (int)ci || !check_small_job(cp.sj[i], *cores[ci], regions[ci])) {
        if (msg) *msg = "small job " + std::to_string(i) + " of circuit " + std::to_string(ci) +
                        " reaches outside its workspace region";
        return false;
      }
  }
  return true;
}

// Records the forward and backward sequences of every circuit.  ws_off[c] is
// circuit c's offset in the batch workspace (> 0).
inline void record_programs(const std::vector<const PlanCore*>& cores, const std::vector<PlanPtrs>& ptrs,
                            const std::vector<uint64_t>& ws_off, std::vector<CircProgram>* fwd,
                            std::vector<CircProgram>* bwd) {
  const size_t n = cores.size();
  fwd->assign(n, CircProgram{});
  bwd->assign(n, CircProgram{});
  for (size_t ci = 0; ci < n; ++ci) {
    const PlanCore& c = *cores[ci];
    char* ws = reinterpret_cast<char*>((uintptr_t)ws_off[ci]);
    RecordExec rf(c, ptrs[ci], (int)ci, (*fwd)[ci]);
    run_forward_fused(c, rf, nullptr, nullptr, nullptr, ws);
    RecordExec rb(c, ptrs[ci], (int)ci, (*bwd)[ci]);
    rb.cp = coef_ptrs(c, ws);
    run_backward_fused(c, rb, nullptr, nullptr, nullptr, nullptr, nullptr, ws);
  }
}

}  // namespace qf
