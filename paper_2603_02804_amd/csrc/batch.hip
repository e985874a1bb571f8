// batch.hip -- mixed batches of circuits on one device: merged launch kernels
// and the qf_batch_* entry points of the C-ABI (include/qfuse.h).
//
//   k_pass_multi<R, NT, BWD>  the fused pass of several circuits in one launch:
//                             each workgroup finds its job (one circuit's pass
//                             launch) by binary search over the jobs' first
//                             blocks, rebases the job's workspace offsets on the
//                             batch workspace and runs the same pass body as
//                             k_pass with its block index inside the job.
//   k_small_multi             the coefficient, assembly and reduction kernels of
//                             several circuits in one launch, same scheme.
// The computation of every circuit is the one of its own plan (Sec. 3.2-3.4);
// merging changes which launch runs a workgroup, not what it computes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "batch.hpp"
#include "device.hpp"
#include "small_kernels.hpp"
#include "gpu_plan.hpp"

namespace qf {

// Workgroups are dealt to the 8 XCDs of the device round-robin by block index.
// The merged launches renumber them so that each XCD runs one contiguous range
// of blocks, i.e. whole jobs of a few circuits: each XCD's L2 (and its CUs'
// scalar caches) then hold the tables of those circuits only.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, n = gridDim.x;
  const int q = n / kXcds, r = n % kXcds, x = b % kXcds;
  return x * q + min(x, r) + b / kXcds;
}

// Last job whose first block is <= b (jobs sorted by first block).
__device__ __forceinline__ int find_job(const int32_t* start, int n_jobs, int b) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cld(start + mid) <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class T>
__device__ __forceinline__ T* rebase(T* p, char* ws) {
  return p ? reinterpret_cast<T*>(ws + reinterpret_cast<uintptr_t>(p)) : p;
}

template <int R, int NT, bool BWD>
__global__ __launch_bounds__(NT, (pass_min_waves<R, BWD>())) void k_pass_multi(const PassJob* jobs, const int32_t* start, int n_jobs,
                                                   char* ws, const CircPtrs* ptrs) {
  const int b = xcd_block();
  const int j = find_job(start, n_jobs, b);
  KArgs A = cld(&jobs[j].A);
  const int circ = cld(&jobs[j].circ);
  A.coef_sh = rebase(A.coef_sh, ws);
  A.coef_ps = rebase(A.coef_ps, ws);
  A.ev_sh = rebase(A.ev_sh, ws);
  A.ev_ps = rebase(A.ev_ps, ws);
  A.src0 = rebase(A.src0, ws);
  A.src1 = rebase(A.src1, ws);
  A.dst = rebase(A.dst, ws);
  A.dst2 = rebase(A.dst2, ws);
  A.dpsi = rebase(A.dpsi, ws);
  A.partF = rebase(A.partF, ws);
  A.partE = rebase(A.partE, ws);
  A.dE = cld(&ptrs[circ].dE);
  pass_body<R, NT, BWD>(A, b - cld(start + j));
}

__global__ __launch_bounds__(kSmallThreads) void k_small_multi(const SmallJob* jobs, const int32_t* start,
                                                               int n_jobs, char* ws, const CircPtrs* ptrs) {
  extern __shared__ double fsum[];
  const int b = xcd_block();
  const int j = find_job(start, n_jobs, b);
  const int kind = cld(&jobs[j].kind);
  const CircPtrs P = cld(&ptrs[cld(&jobs[j].circ)]);
  const int blk = b - cld(start + j);
  const long long idx = (long long)blk * blockDim.x + threadIdx.x;
  switch (kind) {
    case SJ_COEF: {
      CoefArgs a = cld(&jobs[j].u.coef);
      a.theta = P.theta;
      a.x = P.x;
      a.csh = rebase(a.csh, ws);
      a.cps = rebase(a.cps, ws);
      coef_body(a, idx);
      break;
    }
    case SJ_EVENT: {
      EventArgs a = cld(&jobs[j].u.ev);
      a.csh = rebase(a.csh, ws);
      a.cps = rebase(a.cps, ws);
      a.esh = rebase(a.esh, ws);
      a.eps = rebase(a.eps, ws);
      event_body(a, idx);
      break;
    }
    case SJ_REDUCE_E: {
      ReduceEArgs a = cld(&jobs[j].u.re);
      a.partE = rebase(a.partE, ws);
      a.E = P.E;
      reduce_E_body(a, idx);
      break;
    }
    case SJ_ASSEMBLE: {
      AssembleArgs a = cld(&jobs[j].u.as);
      a.theta = P.theta;
      a.x = P.x;
      a.partF = rebase(a.partF, ws);
      a.Gr = rebase(a.Gr, ws);
      assemble_body(a, blk, fsum);
      break;
    }
    case SJ_REDUCE_G: {
      ReduceGArgs a = cld(&jobs[j].u.rg);
      a.Gr = rebase(a.Gr, ws);
      a.dtheta = P.dtheta;
      a.dx = P.dx;
      reduce_grads_body(a, blk, (int)threadIdx.x, fsum);
      break;
    }
    default:
      break;
  }
}

using MultiPassFn = void (*)(const PassJob*, const int32_t*, int, char*, const CircPtrs*);

template <int R, int NT>
static MultiPassFn multi_fn(bool bwd) {
  return bwd ? k_pass_multi<R, NT, true> : k_pass_multi<R, NT, false>;
}

// The same tile shapes as the single-plan pass kernels.
static MultiPassFn select_multi(int cls) {
  if (cls < 0 || cls >= kPassClasses) return nullptr;
  const int R = class_R(cls), NT = class_NT(cls);
  const bool bwd = class_bwd(cls);
  if (R == 5) {
    if (NT == 64) return multi_fn<5, 64>(bwd);
    if (NT == 128) return multi_fn<5, 128>(bwd);
    if (NT == 256) return multi_fn<5, 256>(bwd);
    return nullptr;
  }
  if (R == 4) {
    if (NT == 128) return multi_fn<4, 128>(bwd);
    if (NT == 256) return multi_fn<4, 256>(bwd);
  }
  if (NT != 64) return nullptr;
  switch (R) {
    case 1: return multi_fn<1, 64>(bwd);
    case 2: return multi_fn<2, 64>(bwd);
    case 3: return multi_fn<3, 64>(bwd);
    case 4: return multi_fn<4, 64>(bwd);
    default: return nullptr;
  }
}

// A merged program's job tables on the device.
struct DevProgram {
  char* blob = nullptr;
  const PassJob* pjobs = nullptr;
  const int32_t* pstart = nullptr;
  const SmallJob* sjobs = nullptr;
  const int32_t* sstart = nullptr;
};

static qf_status upload_program(const Program& P, DevProgram* d, std::string* msg) {
  std::vector<char> blob;
  std::vector<size_t> o;
  push_table(blob, o, P.pjobs);
  push_table(blob, o, P.pstart);
  push_table(blob, o, P.sjobs);
  push_table(blob, o, P.sstart);
  if (hipMalloc(&d->blob, blob.size()) != hipSuccess) {
    *msg = "hipMalloc of merged launch tables failed";
    return QF_ERR_OOM;
  }
  if (hipMemcpy(d->blob, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
    *msg = "hipMemcpy of merged launch tables failed";
    return QF_ERR_DEVICE;
  }
  d->pjobs = (const PassJob*)(d->blob + o[0]);
  d->pstart = (const int32_t*)(d->blob + o[1]);
  d->sjobs = (const SmallJob*)(d->blob + o[2]);
  d->sstart = (const int32_t*)(d->blob + o[3]);
  return QF_OK;
}

// Streams and events that let the groups of a program run concurrently: group 0
// runs on the caller's stream, group g > 0 on side[g - 1], forked from and joined
// back into the caller's stream (also inside a graph capture, where the fork
// and join become graph dependencies).
struct GroupStreams {
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
};

static hipError_t launch_program(const Program& P, const DevProgram& d, char* ws, const CircPtrs* ptrs,
                                 hipStream_t st, const GroupStreams& gs) {
  const int G = P.groups;
  if (G > 1 && (int)gs.side.size() < G - 1) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  if (G > 1) {
    if ((e = hipEventRecord(gs.fork, st)) != hipSuccess) return e;
    for (int g = 1; g < G; ++g)
      if ((e = hipStreamWaitEvent(gs.side[g - 1], gs.fork, 0)) != hipSuccess) return e;
  }
  for (const MergedLaunch& L : P.launches) {
    hipStream_t s = L.group == 0 ? st : gs.side[L.group - 1];
    if (L.cls >= 0) {
      MultiPassFn fn = select_multi(L.cls);
      hipLaunchKernelGGL(fn, dim3(L.blocks), dim3(class_NT(L.cls)), L.shmem, s, d.pjobs + L.job0,
                         d.pstart + L.job0, L.n_jobs, ws, ptrs);
    } else {
      hipLaunchKernelGGL(k_small_multi, dim3(L.blocks), dim3(kSmallThreads), L.shmem, s, d.sjobs + L.job0,
                         d.sstart + L.job0, L.n_jobs, ws, ptrs);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int g = 1; g < G; ++g) {
    if ((e = hipEventRecord(gs.join[g - 1], gs.side[g - 1])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st, gs.join[g - 1], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Forward / backward state of one direction of a batch.
struct Direction {
  Program prog;
  DevProgram dev;
  CircPtrs* d_ptrs = nullptr;        // device table, rewritten before every call
  CircPtrs* h_ptrs = nullptr;        // pinned staging of the table
  hipEvent_t copied = nullptr;       // the staging buffer may be rewritten after this
  bool pending = false;
  hipGraphExec_t graph = nullptr;
  char* graph_ws = nullptr;          // workspace address the graph was captured with
};

}  // namespace qf

using namespace qf;

struct qf_batch {
  std::vector<qf_plan*> plans;
  std::vector<int32_t> samples;
  std::vector<uint64_t> ws_off;
  size_t ws_bytes = 0;
  Direction dir[2];                  // 0 forward, 1 backward
  hipStream_t capture = nullptr;     // private stream for graph capture only
  GroupStreams gs;                   // side streams of the concurrent groups
  int mode = QF_LAUNCH_GRAPH;
  int device = 0;
  qf_batch_info info{};
};

static void destroy_batch(qf_batch* b) {
  for (Direction& d : b->dir) {
    if (d.pending && d.copied) (void)hipEventSynchronize(d.copied);
    if (d.graph) (void)hipGraphExecDestroy(d.graph);
    if (d.copied) (void)hipEventDestroy(d.copied);
    if (d.h_ptrs) (void)hipHostFree(d.h_ptrs);
    if (d.d_ptrs) (void)hipFree(d.d_ptrs);
    if (d.dev.blob) (void)hipFree(d.dev.blob);
  }
  if (b->capture) (void)hipStreamDestroy(b->capture);
  for (hipStream_t s : b->gs.side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->gs.join) (void)hipEventDestroy(e);
  if (b->gs.fork) (void)hipEventDestroy(b->gs.fork);
  for (qf_plan* p : b->plans) qf_plan_destroy(p);
  delete b;
}

extern "C" {

qf_status qf_batch_create(const qf_circuit* const* circuits, const int32_t* samples, int32_t n_circuits,
                          const qf_tuning* tuning, qf_batch** out) {
  if (!out) return set_error(QF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!circuits || !samples || n_circuits < 1) return set_error(QF_ERR_INVALID_ARG, "empty batch");
  if (tuning && tuning->mode != 0) return set_error(QF_ERR_UNSUPPORTED, "mixed batches run the fused path only");
  for (int i = 0; i < n_circuits; ++i) {
    if (!circuits[i]) return set_error(QF_ERR_INVALID_ARG, "circuit " + std::to_string(i) + " is NULL");
    if (samples[i] < 1) return set_error(QF_ERR_INVALID_ARG, "samples must be >= 1");
  }
  qf_batch* b = nullptr;
  try {
    b = new qf_batch;
  } catch (...) {
    return set_error(QF_ERR_OOM, "host allocation failed");
  }
  hipGetDevice(&b->device);
  b->samples.assign(samples, samples + n_circuits);
  // merged launches step every circuit pass by pass, so by default no
  // end-of-pass epoch waits for the next pass (fewer passes, fewer steps)
  qf_tuning bt;
  std::memset(&bt, 0, sizeof(bt));
  bt.store_ckpt = -1;
  if (tuning) bt = *tuning;
  for (int i = 0; i < n_circuits; ++i) {
    qf_plan* p = nullptr;
    const qf_tuning ct = batch_plan_tuning(bt, circuits[i]->c.n);
    const qf_status st = qf_plan_create(circuits[i], samples[i], &ct, &p);
    if (st != QF_OK) {
      const std::string m = "circuit " + std::to_string(i) + ": " + qf_last_error();
      destroy_batch(b);
      return set_error(st, m);
    }
    b->plans.push_back(p);
    if (p->core.S.general_obs) {
      destroy_batch(b);
      return set_error(QF_ERR_UNSUPPORTED, "circuit " + std::to_string(i) +
                                               ": mixed batches take Z-string observables only");
    }
  }
  std::string msg;
  qf_status st = QF_OK;
  try {
    std::vector<const PlanCore*> cores;
    std::vector<PlanPtrs> ptrs;
    for (qf_plan* p : b->plans) {
      cores.push_back(&p->core);
      ptrs.push_back(p->dev.p);
    }
    b->ws_bytes = batch_layout(cores, &b->ws_off);
    std::vector<Region> regions;
    for (int i = 0; i < n_circuits; ++i) regions.push_back({b->ws_off[i], b->ws_off[i] + cores[i]->ws_bytes});
    std::vector<CircProgram> fwd, bwd;
    record_programs(cores, ptrs, b->ws_off, &fwd, &bwd);
    if (!check_program(fwd, cores, regions, &msg) || !check_program(bwd, cores, regions, &msg)) {
      st = QF_ERR_INTERNAL;
    }
    const std::vector<int> order = batch_order(cores);
    if (st == QF_OK && (!merge_grouped(fwd, cores, order, &b->dir[0].prog, &msg) ||
                        !merge_grouped(bwd, cores, order, &b->dir[1].prog, &msg)))
      st = QF_ERR_UNSUPPORTED;
    for (int k = 0; st == QF_OK && k < 2; ++k)
      for (const MergedLaunch& L : b->dir[k].prog.launches)
        if (L.cls >= 0 && !select_multi(L.cls)) {
          st = QF_ERR_UNSUPPORTED;
          msg = "no merged pass kernel for a circuit's tile shape";
          break;
        }
  } catch (const std::exception& e) {
    st = QF_ERR_INTERNAL;
    msg = e.what();
  }
  for (int k = 0; st == QF_OK && k < 2; ++k) {
    Direction& d = b->dir[k];
    st = upload_program(d.prog, &d.dev, &msg);
    if (st != QF_OK) break;
    const size_t tb = sizeof(CircPtrs) * n_circuits;
    if (hipMalloc(&d.d_ptrs, tb) != hipSuccess || hipHostMalloc(&d.h_ptrs, tb, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&d.copied, hipEventDisableTiming) != hipSuccess) {
      st = QF_ERR_OOM;
      msg = "allocation of the pointer tables failed";
    }
  }
  if (st == QF_OK && hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) {
    st = QF_ERR_DEVICE;
    msg = "hipStreamCreateWithFlags failed";
  }
  // one side stream (default priority) and join event per group after the first
  const int groups = std::max(b->dir[0].prog.groups, b->dir[1].prog.groups);
  if (st == QF_OK && groups > 1) {
    if (hipEventCreateWithFlags(&b->gs.fork, hipEventDisableTiming) != hipSuccess) st = QF_ERR_DEVICE;
    for (int g = 1; st == QF_OK && g < groups; ++g) {
      hipStream_t s = nullptr;
      hipEvent_t e = nullptr;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        st = QF_ERR_DEVICE;
        break;
      }
      b->gs.side.push_back(s);
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        st = QF_ERR_DEVICE;
        break;
      }
      b->gs.join.push_back(e);
    }
    if (st != QF_OK) msg = "creation of the group streams failed";
  }
  if (st != QF_OK) {
    destroy_batch(b);
    return set_error(st, msg);
  }
  // accounting
  qf_batch_info& I = b->info;
  I.n_circuits = n_circuits;
  for (int i = 0; i < n_circuits; ++i) {
    qf_plan_info pi;
    qf_plan_get_info(b->plans[i], &pi);
    I.samples += samples[i];
    I.fwd_bytes += pi.fwd_bytes_per_sample * samples[i];
    I.bwd_bytes += pi.bwd_bytes_per_sample * samples[i];
    I.fwd_flops += pi.fwd_flops_per_sample * samples[i];
    I.bwd_flops += pi.bwd_flops_per_sample * samples[i];
  }
  I.fwd_steps = b->dir[0].prog.steps;
  I.bwd_steps = b->dir[1].prog.steps;
  I.fwd_launches = (int64_t)b->dir[0].prog.launches.size();
  I.bwd_launches = (int64_t)b->dir[1].prog.launches.size();
  I.fwd_jobs = b->dir[0].prog.jobs;
  I.bwd_jobs = b->dir[1].prog.jobs;
  *out = b;
  return QF_OK;
}

qf_status qf_batch_destroy(qf_batch* b) {
  if (b) destroy_batch(b);
  return QF_OK;
}

qf_status qf_batch_get_info(const qf_batch* b, qf_batch_info* info) {
  if (!b || !info) return set_error(QF_ERR_INVALID_ARG, "NULL argument");
  *info = b->info;
  return QF_OK;
}

qf_status qf_batch_workspace_size(const qf_batch* b, size_t* bytes) {
  if (!b || !bytes) return set_error(QF_ERR_INVALID_ARG, "NULL argument");
  *bytes = b->ws_bytes;
  return QF_OK;
}

qf_status qf_batch_set_launch_mode(qf_batch* b, int32_t mode) {
  if (!b) return set_error(QF_ERR_INVALID_ARG, "batch is NULL");
  if (mode < QF_LAUNCH_GRAPH || mode > QF_LAUNCH_PER_CIRCUIT) return set_error(QF_ERR_INVALID_ARG, "unknown mode");
  b->mode = mode;
  return QF_OK;
}

}  // extern "C"

namespace {

qf_status check_batch_call(qf_batch* b, void* ws, size_t ws_bytes) {
  if (!b) return set_error(QF_ERR_INVALID_ARG, "batch is NULL");
  if (!ws || ws_bytes < b->ws_bytes)
    return set_error(QF_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, batch needs " +
                                           std::to_string(b->ws_bytes));
  if (((uintptr_t)ws & 255) != 0) return set_error(QF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  int dev = -1;
  hipGetDevice(&dev);
  if (dev != b->device) return set_error(QF_ERR_INVALID_ARG, "batch was created on another device");
  return QF_OK;
}

// Writes the pointer table of direction k and enqueues its upload on st.
qf_status stage_pointers(qf_batch* b, int k, const std::vector<CircPtrs>& tab, hipStream_t st) {
  Direction& d = b->dir[k];
  if (d.pending && hipEventSynchronize(d.copied) != hipSuccess)
    return set_error(QF_ERR_DEVICE, "hipEventSynchronize failed");
  std::copy(tab.begin(), tab.end(), d.h_ptrs);
  if (hipMemcpyAsync(d.d_ptrs, d.h_ptrs, sizeof(CircPtrs) * tab.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventRecord(d.copied, st) != hipSuccess)
    return set_error(QF_ERR_DEVICE, "upload of the pointer table failed");
  d.pending = true;
  return QF_OK;
}

qf_status run_merged(qf_batch* b, int k, char* ws, hipStream_t st) {
  Direction& d = b->dir[k];
  if (b->mode == QF_LAUNCH_MERGED) {
    const hipError_t e = launch_program(d.prog, d.dev, ws, d.d_ptrs, st, b->gs);
    if (e != hipSuccess) return set_error(QF_ERR_DEVICE, std::string("merged launch: ") + hipGetErrorString(e));
    return QF_OK;
  }
  if (!d.graph || d.graph_ws != ws) {
    if (d.graph) {
      (void)hipGraphExecDestroy(d.graph);
      d.graph = nullptr;
    }
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(QF_ERR_DEVICE, "hipStreamBeginCapture failed");
    const hipError_t e = launch_program(d.prog, d.dev, ws, d.d_ptrs, b->capture, b->gs);
    const hipError_t e2 = hipStreamEndCapture(b->capture, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return set_error(QF_ERR_DEVICE, "graph capture of the merged launches failed");
    }
    const hipError_t e3 = hipGraphInstantiate(&d.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
      d.graph = nullptr;
      return set_error(QF_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    d.graph_ws = ws;
  }
  if (hipGraphLaunch(d.graph, st) != hipSuccess) return set_error(QF_ERR_DEVICE, "hipGraphLaunch failed");
  return QF_OK;
}

}  // namespace

extern "C" {

qf_status qf_batch_forward(qf_batch* b, const float* const* theta, const float* const* x, float* const* E,
                           void* ws, size_t ws_bytes, void* stream) {
  qf_status st = check_batch_call(b, ws, ws_bytes);
  if (st != QF_OK) return st;
  if (!theta || !E) return set_error(QF_ERR_INVALID_ARG, "NULL pointer array");
  const int n = (int)b->plans.size();
  std::vector<CircPtrs> tab(n);
  for (int i = 0; i < n; ++i) {
    const Circuit& C = b->plans[i]->core.C;
    const float* xi = x ? x[i] : nullptr;
    if (!E[i] || (C.P > 0 && !theta[i]) || (C.F > 0 && !xi))
      return set_error(QF_ERR_INVALID_ARG, "NULL buffer for circuit " + std::to_string(i));
    tab[i] = CircPtrs{theta[i], xi, E[i], nullptr, nullptr, nullptr};
  }
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  if (b->mode == QF_LAUNCH_PER_CIRCUIT) {
    for (int i = 0; i < n; ++i) {
      st = qf_forward(b->plans[i], tab[i].theta, tab[i].x, tab[i].E, w + b->ws_off[i], b->plans[i]->core.ws_bytes,
                      stream);
      if (st != QF_OK) return st;
    }
    return QF_OK;
  }
  st = stage_pointers(b, 0, tab, s);
  if (st != QF_OK) return st;
  return run_merged(b, 0, w, s);
}

qf_status qf_batch_backward(qf_batch* b, const float* const* theta, const float* const* x, const float* const* dE,
                            float* const* dtheta, float* const* dx, void* ws, size_t ws_bytes, void* stream) {
  qf_status st = check_batch_call(b, ws, ws_bytes);
  if (st != QF_OK) return st;
  if (!theta || !dE || !dtheta) return set_error(QF_ERR_INVALID_ARG, "NULL pointer array");
  const int n = (int)b->plans.size();
  std::vector<CircPtrs> tab(n);
  for (int i = 0; i < n; ++i) {
    const Circuit& C = b->plans[i]->core.C;
    const float* xi = x ? x[i] : nullptr;
    if (!dE[i] || (C.P > 0 && (!theta[i] || !dtheta[i])) || (C.F > 0 && !xi))
      return set_error(QF_ERR_INVALID_ARG, "NULL buffer for circuit " + std::to_string(i));
    tab[i] = CircPtrs{theta[i], xi, nullptr, dE[i], dtheta[i], dx ? dx[i] : nullptr};
  }
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  if (b->mode == QF_LAUNCH_PER_CIRCUIT) {
    for (int i = 0; i < n; ++i) {
      st = qf_backward(b->plans[i], tab[i].theta, tab[i].x, tab[i].dE, tab[i].dtheta, tab[i].dx, w + b->ws_off[i],
                       b->plans[i]->core.ws_bytes, stream);
      if (st != QF_OK) return st;
    }
    return QF_OK;
  }
  st = stage_pointers(b, 1, tab, s);
  if (st != QF_OK) return st;
  return run_merged(b, 1, w, s);
}

}  // extern "C"
