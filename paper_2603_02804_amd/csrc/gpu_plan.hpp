// gpu_plan.hpp -- host-side device objects of the C-ABI: a plan's table blob in
// device memory, launch-time profiling, and the opaque handles of include/qfuse.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "kargs.hpp"

namespace qf {

// A plan's read-only tables, uploaded once into one device allocation.
struct DevPlan {
  char* blob = nullptr;
  size_t bytes = 0;
  PlanPtrs p;
};

template <class T>
inline void push_table(std::vector<char>& blob, std::vector<size_t>& offs, const std::vector<T>& v) {
  size_t off = align_up(blob.size());
  blob.resize(off + std::max<size_t>(sizeof(T), v.size() * sizeof(T)), 0);
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
  offs.push_back(off);
}

// Per-thread bases of every layout, so that the pass kernels read a thread's
// part of an index instead of forming it with one AND-XOR per thread bit: entry
// [layout * NT + t] = {LDS byte offset, logical basis index, memory index} of
// thread t, the XOR of lds_thr[i] (log_thr[i], mem_thr[i]) over the set bits i of t.
inline std::vector<ThrBase> thread_base_table(const Schedule& S) {
  std::vector<ThrBase> tab;
  if (S.NT <= 0) return tab;
  tab.resize(S.layouts.size() * (size_t)S.NT);
  for (size_t l = 0; l < S.layouts.size(); ++l) {
    const LayoutRec& L = S.layouts[l];
    for (int t = 0; t < S.NT; ++t) {
      ThrBase b{0u, 0u, 0u, 0u};
      for (int i = 0; i < kMaxThreadBits; ++i)
        if ((t >> i) & 1) {
          b.lds ^= L.lds_thr[i];
          b.log ^= L.log_thr[i];
          b.mem ^= L.mem_thr[i];
        }
      tab[l * (size_t)S.NT + t] = b;
    }
  }
  return tab;
}

inline qf_status upload_plan(const PlanCore& c, DevPlan* d, std::string* msg) {
  std::vector<char> blob;
  std::vector<size_t> o;
  std::vector<uint32_t> zm;
  for (const qf_pauli& p : c.C.obs) zm.push_back((uint32_t)p.z_mask);
  push_table(blob, o, c.S.ops);          // 0
  push_table(blob, o, c.S.layouts);      // 1
  push_table(blob, o, c.S.czg);          // 2
  push_table(blob, o, c.S.funcs);        // 3
  push_table(blob, o, c.S.passes);       // 4
  push_table(blob, o, zm);               // 5
  push_table(blob, o, c.S.runs);         // 6
  push_table(blob, o, c.S.run_gates);    // 7
  push_table(blob, o, c.S.gates);        // 8
  push_table(blob, o, c.coef_runs_sh);   // 9
  push_table(blob, o, c.coef_runs_ps);   // 10
  push_table(blob, o, c.partF_off);      // 11
  push_table(blob, o, c.seg_runs);       // 12
  push_table(blob, o, c.seg_run_begin);  // 13
  push_table(blob, o, c.th_ref_begin);   // 14
  push_table(blob, o, c.th_refs);        // 15
  push_table(blob, o, c.in_ref_begin);   // 16
  push_table(blob, o, c.in_refs);        // 17
  push_table(blob, o, c.S.pev);          // 18
  push_table(blob, o, c.S.cza);          // 19
  push_table(blob, o, c.S.events);       // 20
  push_table(blob, o, c.S.pass_run_begin);  // 21
  push_table(blob, o, c.S.pass_runs);    // 22
  push_table(blob, o, c.S.rygs);         // 23
  push_table(blob, o, c.S.epochs);       // 24
  push_table(blob, o, c.S.phas);         // 25
  push_table(blob, o, pauli_table(c));   // 26
  push_table(blob, o, c.C.consts);       // 27
  push_table(blob, o, thread_base_table(c.S));   // 28
  d->bytes = blob.size();
  if (hipMalloc(&d->blob, d->bytes) != hipSuccess) {
    if (msg) *msg = "hipMalloc of plan tables failed";
    return QF_ERR_OOM;
  }
  if (hipMemcpy(d->blob, blob.data(), d->bytes, hipMemcpyHostToDevice) != hipSuccess) {
    if (msg) *msg = "hipMemcpy of plan tables failed";
    return QF_ERR_DEVICE;
  }
  char* b = d->blob;
  PlanPtrs& p = d->p;
  p.ops = (const Op*)(b + o[0]);
  p.layouts = (const LayoutRec*)(b + o[1]);
  p.czg = (const CzGroup*)(b + o[2]);
  p.funcs = (const FuncEntry*)(b + o[3]);
  p.passes = (const PassRec*)(b + o[4]);
  p.zmask = (const uint32_t*)(b + o[5]);
  Tabs& t = p.tabs;
  t.runs = (const RunRec*)(b + o[6]);
  t.run_gates = (const int32_t*)(b + o[7]);
  t.gates = (const GateRec*)(b + o[8]);
  t.coef_runs_sh = (const int32_t*)(b + o[9]);
  t.coef_runs_ps = (const int32_t*)(b + o[10]);
  t.passes = p.passes;
  t.partF_off = (const int64_t*)(b + o[11]);
  t.seg_runs = (const int32_t*)(b + o[12]);
  t.seg_run_begin = (const int32_t*)(b + o[13]);
  t.th_ref_begin = (const int32_t*)(b + o[14]);
  t.th_refs = (const int32_t*)(b + o[15]);
  t.in_ref_begin = (const int32_t*)(b + o[16]);
  t.in_refs = (const int32_t*)(b + o[17]);
  p.pev = (const PhaseEv*)(b + o[18]);
  p.cza = (const CzaRec*)(b + o[19]);
  t.events = (const EventRec*)(b + o[20]);
  t.pass_run_begin = (const int32_t*)(b + o[21]);
  t.pass_runs = (const int32_t*)(b + o[22]);
  p.rygs = (const RygEntry*)(b + o[23]);
  p.epochs = (const EpochRec*)(b + o[24]);
  p.phas = (const PhaEntry*)(b + o[25]);
  p.pauli = (const PauliRec*)(b + o[26]);
  t.consts = (const double*)(b + o[27]);
  p.tbases = (const ThrBase*)(b + o[28]);
  return QF_OK;
}

// Event pairs bracketing launches while a plan's profiling is enabled.
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> ev;          // pool, reused across reads
  std::vector<int> kind;               // class of each recorded pair
  size_t used = 0;                     // pairs recorded since the last read
  hipEvent_t get(size_t i) {
    while (ev.size() <= i) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[i];
  }
  void begin(hipStream_t st) {
    if (!on) return;
    hipEvent_t e = get(2 * used);
    if (e) (void)hipEventRecord(e, st);
  }
  void end(hipStream_t st, int k) {
    if (!on) return;
    hipEvent_t e = get(2 * used + 1);
    if (e) (void)hipEventRecord(e, st);
    if (kind.size() <= used) kind.resize(used + 1);
    kind[used++] = k;
  }
  ~Profiler() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// Records the message of the failing C-ABI call and returns its status.
qf_status set_error(qf_status s, const std::string& m);

// True when a pass kernel is compiled for the tile shape.
bool have_pass_kernel(int R, int NT);

}  // namespace qf

struct qf_circuit {
  qf::Circuit c;
};

struct qf_plan {
  qf::PlanCore core;
  qf::DevPlan dev;
  int device = 0;
  qf::Profiler prof;
};
