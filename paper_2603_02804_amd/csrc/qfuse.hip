// qfuse.hip -- gfx950 kernels of one plan, their launch backend and the plan
// entry points of the C-ABI (include/qfuse.h).
//
// Kernels
//   k_pass<R, NT, BWD>  fused pass: one workgroup per (sample, tile of 2^k amplitudes).
//                       Forward (Sec. 3.2): load or initialise the tile, apply the
//                       pass's runs (merged 2x2 matrices) on register-resident qubits,
//                       CZ sign flips from the global basis index (App. B.1), LDS
//                       permutes between register layouts, write once.
//                       Backward (Sec. 3.3): load the stored pass output psi and the
//                       adjoint lambda; for every run in reverse evaluate the three
//                       functionals Im<lambda|P_q|psi> (P = X, Y, Z) at the cut after
//                       the run, then un-apply the run from psi and lambda in
//                       registers; write lambda once.
//   k_coef              merged 2x2 matrix of every run, u(phi) = cos(phi/2) I -
//                       i sin(phi/2) P (Sec. 3.3), multiplied in gate order.
//   k_assemble          per-gate gradients of a run from its functionals:
//                       dL/dtheta_g = Re<lambda_g|du_g|psi_{g-1}> = 1/2 Im<lambda|G_g|psi>
//                       with G_g = K_g P_g K_g^dagger, K_g = later gates of the run.
//   k_reduce_grads      sums over the batch (theta) and over shared angles, fixed order.
//   k_reduce_E          expectation partial sums -> E[b][k] (App. B.2).
//   k_pauli_expect/seed expectations and adjoint seed of general Pauli strings
//                       from a stored state (App. B.2).
//   k_pg_*              one-kernel-per-gate baseline.
// The kernel bodies live in device.hpp, shared with the merged mixed-batch
// kernels of batch.hip.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "small_kernels.hpp"
#include "gpu_plan.hpp"

namespace qf {

template <int R, int NT, bool BWD>
__global__ __launch_bounds__(NT, (pass_min_waves<R, BWD>())) void k_pass(const KArgs A) {
  pass_body<R, NT, BWD>(A, blockIdx.x);
}

template <class Real>
__global__ __launch_bounds__(kSmallThreads) void k_coef(const CoefArgsT<Real> a) {
  coef_body(a, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kSmallThreads) void k_event_coef(const EventArgs a) {
  event_body(a, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kSmallThreads) void k_assemble(const AssembleArgs a) {
  extern __shared__ double fsum[];
  assemble_body(a, blockIdx.x, fsum);
}

template <class Real>
__global__ __launch_bounds__(kSmallThreads) void k_reduce_grads(const ReduceGArgsT<Real> a) {
  __shared__ double red[kSmallThreads];
  reduce_grads_body(a, blockIdx.x, threadIdx.x, red);
}

template <class Real>
__global__ __launch_bounds__(kSmallThreads) void k_reduce_E(const ReduceEArgsT<Real> a) {
  reduce_E_body(a, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// per-gate kernels: the unfused baseline (float) and the complex128
// validation path (double) share them
// ---------------------------------------------------------------------------
template <class Real> struct Cplx;
template <> struct Cplx<float> {
  using T = float2;
  static __device__ __forceinline__ T make(float a, float b) { return make_float2(a, b); }
};
template <> struct Cplx<double> {
  using T = double2;
  static __device__ __forceinline__ T make(double a, double b) { return make_double2(a, b); }
};

__device__ __forceinline__ long long pair_lo(long long p, int q) {
  return ((p >> q) << (q + 1)) | (p & ((1ll << q) - 1));
}

// (x0, x1) <- M (x0, x1) for a 2x2 complex M given row-major as 8 reals
template <class Real, class V>
__device__ __forceinline__ void mat2_apply(const Real (&m)[8], V& x0, V& x1) {
  const V y0 = Cplx<Real>::make(m[0] * x0.x - m[1] * x0.y + m[2] * x1.x - m[3] * x1.y,
                                m[0] * x0.y + m[1] * x0.x + m[2] * x1.y + m[3] * x1.x);
  const V y1 = Cplx<Real>::make(m[4] * x0.x - m[5] * x0.y + m[6] * x1.x - m[7] * x1.y,
                                m[4] * x0.y + m[5] * x0.x + m[6] * x1.y + m[7] * x1.x);
  x0 = y0;
  x1 = y1;
}

template <class Real>
__device__ __forceinline__ const Real* pg_coef_row(const Real* csh, const Real* cps, int ref, int sample, int n_ps) {
  return ref >= 0 ? csh + 8 * (long long)ref : cps + 8 * ((long long)sample * n_ps + (-1 - ref));
}

template <class Real>
__global__ void k_pg_init(typename Cplx<Real>::T* psi, long long amps, int nb) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= amps * nb) return;
  psi[i] = Cplx<Real>::make((i % amps) == 0 ? 1 : 0, 0);
}

template <class Real>
__global__ __launch_bounds__(kPgThreads) void k_pg_rot(typename Cplx<Real>::T* psi, long long amps, int q, int ref,
                                                       int sample0, const Real* csh, const Real* cps, int n_ps,
                                                       int blocks) {
  using V = typename Cplx<Real>::T;
  const int s = blockIdx.x / blocks, blk = blockIdx.x - s * blocks;
  V* v = psi + (long long)s * amps;
  const Real* c = pg_coef_row(csh, cps, ref, sample0 + s, n_ps);
  Real m[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) m[i] = c[i];
  const long long pairs = amps >> 1;
#pragma unroll
  for (int k = 0; k < kPgPairsPerThread; ++k) {
    const long long p = ((long long)blk * kPgPairsPerThread + k) * kPgThreads + threadIdx.x;
    if (p >= pairs) break;
    const long long i0 = pair_lo(p, q), i1 = i0 | (1ll << q);
    V x0 = v[i0], x1 = v[i1];
    mat2_apply(m, x0, x1);
    v[i0] = x0;
    v[i1] = x1;
  }
}

// CZ touches only the quarter of the amplitudes with both bits set.
template <class Real>
__global__ void k_pg_cz(typename Cplx<Real>::T* psi, typename Cplx<Real>::T* lam, long long amps, int qa, int qb,
                        int nb) {
  using V = typename Cplx<Real>::T;
  const long long quarter = amps >> 2;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= quarter * nb) return;
  const long long s = idx / quarter, j = idx - s * quarter;
  const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
  long long i = pair_lo(j, lo);
  i = pair_lo(i, hi);
  i |= (1ll << lo) | (1ll << hi);
  V* v = psi + s * amps + i;
  *v = Cplx<Real>::make(-v->x, -v->y);
  if (lam) {
    V* w = lam + s * amps + i;
    *w = Cplx<Real>::make(-w->x, -w->y);
  }
}

// Block sum of NV per-thread values; writes the first `count` sums to out[0..count).
template <int NV, class Real>
__device__ inline void block_reduce(Real (&v)[NV], Real* out, int count) {
  __shared__ Real sm[NV][kPgThreads / 64];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    Real x = v[k];
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
    if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < NV && (int)threadIdx.x < count) {
    Real acc = 0;
    for (int w = 0; w < kPgThreads / 64; ++w) acc += sm[threadIdx.x][w];
    out[threadIdx.x] = acc;
  }
}

// i^ny * z
template <class V>
__device__ __forceinline__ V mul_i_pow(V z, int ny) {
  V r = z;
  if (ny & 1) { r.x = -z.y; r.y = z.x; }
  if (ny & 2) { r.x = -r.x; r.y = -r.y; }
  return r;
}

// Pauli-string expectations (App. B.2): per block, partial sums over its
// amplitudes y of Re conj(psi_y) (P_k psi)_y with (P psi)_y =
// i^ny (-1)^{popcount((y ^ xm) & zm)} psi_{y ^ xm}.  The masks are in the bit
// order of the stored state.  Blocks of one sample: `blocks`.
template <class Real>
__global__ __launch_bounds__(kPgThreads) void k_pauli_expect(const typename Cplx<Real>::T* psi, long long stride,
                                                             long long amps, int K, const PauliRec* obs, Real* partE,
                                                             int blocks) {
  using V = typename Cplx<Real>::T;
  const int s = blockIdx.x / blocks, blk = blockIdx.x - s * blocks;
  const V* v = psi + (long long)s * stride;
  for (int k0 = 0; k0 < K; k0 += 8) {
    Real acc[8];
    for (int k = 0; k < 8; ++k) acc[k] = 0;
    for (int k2 = 0; k2 < kPauliAmpsPerThread; ++k2) {
      const long long y = ((long long)blk * kPauliAmpsPerThread + k2) * kPgThreads + threadIdx.x;
      if (y >= amps) break;
      const V a = v[y];
      for (int k = 0; k < 8; ++k) {
        if (k0 + k >= K) break;
        const PauliRec o = obs[k0 + k];
        const long long yx = y ^ (long long)o.xm;
        const V b = v[yx];
        // conj(a) * b, times i^ny, real part, times the sign
        V c;
        c.x = a.x * b.x + a.y * b.y;
        c.y = a.x * b.y - a.y * b.x;
        const Real re = mul_i_pow(c, o.ny).x;
        acc[k] += (__popcll((unsigned long long)(yx & (long long)o.zm)) & 1) ? -re : re;
      }
    }
    block_reduce<8>(acc, partE + ((long long)s * blocks + blk) * K + k0, K - k0);
    __syncthreads();
  }
}

// Adjoint seed lambda = 2 sum_k g_k P_k psi (eq. bwd_exp_val with the chain
// rule), one thread per amplitude.
template <class Real>
__global__ void k_pauli_seed(const typename Cplx<Real>::T* psi, long long psi_stride, typename Cplx<Real>::T* lam,
                             long long lam_stride, long long amps, int nb, int sample0, int K, const PauliRec* obs,
                             const Real* dE) {
  using V = typename Cplx<Real>::T;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= amps * nb) return;
  const long long s = idx / amps, y = idx - s * amps;
  const V* v = psi + s * psi_stride;
  V acc = Cplx<Real>::make(0, 0);
  for (int k = 0; k < K; ++k) {
    const PauliRec o = obs[k];
    const long long yx = y ^ (long long)o.xm;
    const Real g = dE[(sample0 + s) * K + k];
    const Real w = (__popcll((unsigned long long)(yx & (long long)o.zm)) & 1) ? -g : g;
    const V t = mul_i_pow(v[yx], o.ny);
    acc.x += w * t.x;
    acc.y += w * t.y;
  }
  lam[s * lam_stride + y] = Cplx<Real>::make(2 * acc.x, 2 * acc.y);
}

// Backward of one gate: the functionals Im<lambda|P|psi> (P = X, Y, Z) at the
// cut after the gate, then psi <- u^dagger psi and lambda <- u^dagger lambda.
template <class Real>
__global__ __launch_bounds__(kPgThreads) void k_pg_rot_bwd(typename Cplx<Real>::T* psi, typename Cplx<Real>::T* lam,
                                                           long long amps, int q, int ref, int sample0,
                                                           const Real* csh, const Real* cps, int n_ps, int blocks,
                                                           int chunk, int slot, Real* partF) {
  using V = typename Cplx<Real>::T;
  const int s = blockIdx.x / blocks, blk = blockIdx.x - s * blocks;
  V* v = psi + (long long)s * amps;
  V* w = lam + (long long)s * amps;
  const Real* c = pg_coef_row(csh, cps, ref, sample0 + s, n_ps);
  // u^dagger: transpose and conjugate
  const Real m[8] = {c[0], -c[1], c[4], -c[5], c[2], -c[3], c[6], -c[7]};
  const long long pairs = amps >> 1;
  Real f[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < kPgPairsPerThread; ++k) {
    const long long p = ((long long)blk * kPgPairsPerThread + k) * kPgThreads + threadIdx.x;
    if (p >= pairs) break;
    const long long i0 = pair_lo(p, q), i1 = i0 | (1ll << q);
    V p0 = v[i0], p1 = v[i1], l0 = w[i0], l1 = w[i1];
    f[0] += l0.x * p1.y - l0.y * p1.x + l1.x * p0.y - l1.y * p0.x;
    f[1] += (l1.x * p0.x + l1.y * p0.y) - (l0.x * p1.x + l0.y * p1.y);
    f[2] += (l0.x * p0.y - l0.y * p0.x) - (l1.x * p1.y - l1.y * p1.x);
    mat2_apply(m, p0, p1);
    mat2_apply(m, l0, l1);
    v[i0] = p0;
    v[i1] = p1;
    w[i0] = l0;
    w[i1] = l1;
  }
  block_reduce<3>(f, partF + (((long long)s * chunk + slot) * blocks + blk) * 3, 3);
}

template <class Real>
__global__ void k_pg_assemble(Tabs T, int r0, int cnt, int nb, int chunk, int blocks, int n_angle,
                              const Real* theta, const Real* x, int F, int sample0, const Real* partF, Real* Gr) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)cnt * nb) return;
  const int s = (int)(idx / cnt), i = (int)(idx - (long long)s * cnt);
  const int r = r0 + i, slot = r % chunk;
  double f[3] = {0, 0, 0};
  for (int b = 0; b < blocks; ++b)
    for (int P = 0; P < 3; ++P) f[P] += partF[(((long long)s * chunk + slot) * blocks + b) * 3 + P];
  run_grads(T, r, theta, x, F, sample0 + s, f[0], f[1], f[2], Gr + (long long)s * n_angle, 0);
}

// ---------------------------------------------------------------------------
// launch backend of one plan
// ---------------------------------------------------------------------------
using PassFn = void (*)(const KArgs);

template <int R, int NT, bool BWD>
static PassFn pass_fn() {
  return k_pass<R, NT, BWD>;
}

static PassFn select_pass(int R, int NT, bool bwd) {
  if (R == 5) {
    if (NT == 64) return bwd ? pass_fn<5, 64, true>() : pass_fn<5, 64, false>();
    if (NT == 128) return bwd ? pass_fn<5, 128, true>() : pass_fn<5, 128, false>();
    if (NT == 256) return bwd ? pass_fn<5, 256, true>() : pass_fn<5, 256, false>();
    return nullptr;
  }
  if (R == 4) {
    if (NT == 128) return bwd ? pass_fn<4, 128, true>() : pass_fn<4, 128, false>();
    if (NT == 256) return bwd ? pass_fn<4, 256, true>() : pass_fn<4, 256, false>();
  }
  if (NT != 64) return nullptr;
  switch (R) {
    case 1: return bwd ? pass_fn<1, 64, true>() : pass_fn<1, 64, false>();
    case 2: return bwd ? pass_fn<2, 64, true>() : pass_fn<2, 64, false>();
    case 3: return bwd ? pass_fn<3, 64, true>() : pass_fn<3, 64, false>();
    case 4: return bwd ? pass_fn<4, 64, true>() : pass_fn<4, 64, false>();
    default: return nullptr;
  }
}

bool have_pass_kernel(int R, int NT) { return select_pass(R, NT, false) != nullptr; }

struct GpuExec {
  const PlanCore& c;
  const DevPlan& d;
  hipStream_t st;
  Profiler* prof = nullptr;
  void pb() { if (prof) prof->begin(st); }
  void pe(int k) { if (prof) prof->end(st, k); }
  const float* theta = nullptr;
  const float* x = nullptr;
  CoefPtrs cp;
  qf_status err = QF_OK;
  std::string msg;
  GpuExec(const PlanCore& pc, const DevPlan& dp, hipStream_t s) : c(pc), d(dp), st(s) {}

  void check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && err == QF_OK) {
      err = QF_ERR_DEVICE;
      msg = std::string(what) + ": " + hipGetErrorString(e);
    }
  }
  qf_status status() const { return err; }

  void coef(const float* th, const float* xx, char* ws) {
    theta = th;
    x = xx;
    cp = coef_ptrs(c, ws);
    const CoefArgs a = make_coef_args(c, d.p, th, xx, cp);
    if (coef_items(a) > 0) {
      pb();
      hipLaunchKernelGGL(k_coef<float>, dim3(blocks_for(coef_items(a))), dim3(kSmallThreads), 0, st, a);
      pe(2);
      check("k_coef");
    }
    const EventArgs e = make_event_args(c, d.p, cp);
    if (event_items(e) > 0) {
      pb();
      hipLaunchKernelGGL(k_event_coef, dim3(blocks_for(event_items(e))), dim3(kSmallThreads), 0, st, e);
      pe(2);
      check("k_event_coef");
    }
  }

  void pass(const PassLaunch& L) {
    const Schedule& S = c.S;
    PassFn fn = select_pass(S.R, S.NT, L.bwd);
    if (!fn) {
      if (err == QF_OK) { err = QF_ERR_UNSUPPORTED; msg = "no pass kernel for this tile shape"; }
      return;
    }
    const KArgs A = make_pass_args(c, d.p, cp, L);
    pb();
    hipLaunchKernelGGL(fn, dim3(pass_blocks(c, L.nb)), dim3(S.NT), pass_shmem(c, L.bwd), st, A);
    pe(L.bwd ? 1 : 0);
    check(L.bwd ? "k_pass(bwd)" : "k_pass(fwd)");
  }

  void reduce_E(int nb, int sample0, const float* partE, float* E) {
    const ReduceEArgs a = make_reduce_E_args<float>(c, nb, sample0, c.tiles * c.waves, partE, E);
    pb();
    hipLaunchKernelGGL(k_reduce_E<float>, dim3(blocks_for((long long)nb * c.C.K)), dim3(kSmallThreads), 0, st, a);
    pe(2);
    check("k_reduce_E");
  }

  void assemble(int seg, int nb, int sample0, const float* th, const float* xx, const float* partF, float* Gr) {
    const AssembleArgs a = make_assemble_args(c, d.p, seg, nb, sample0, th, xx, partF, Gr);
    if (a.np == 0 || nb == 0) return;
    pb();
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)(nb * a.np)), dim3(kSmallThreads), assemble_shmem(c), st, a);
    pe(2);
    check("k_assemble");
  }

  void reduce_grads(int nb, int sample0, const float* Gr, float* dtheta, float* dx, bool accumulate) {
    const ReduceGArgs a = make_reduce_grads_args<float>(c, d.p, nb, sample0, Gr, dtheta, dx, accumulate);
    if (a.P == 0 && a.dx_items() == 0) return;
    pb();
    hipLaunchKernelGGL(k_reduce_grads<float>, dim3((unsigned)reduce_grads_blocks(a)), dim3(kSmallThreads), 0, st, a);
    pe(2);
    check("k_reduce_grads");
  }

  // per-gate kernels, in float (baseline) or double (complex128 validation)
  template <class Real>
  using V = typename Cplx<Real>::T;
  template <class Real>
  void pg_coef(const Real* th, const Real* xx, char* ws) {
    const CoefArgsT<Real> a =
        make_coef_args_t<Real>(c, d.p, th, xx, at<Real>(ws, c.off_coef_sh), at<Real>(ws, c.off_coef_ps));
    if (coef_items(a) == 0) return;
    pb();
    hipLaunchKernelGGL(k_coef<Real>, dim3(blocks_for(coef_items(a))), dim3(kSmallThreads), 0, st, a);
    pe(2);
    check("k_coef");
  }
  template <class Real>
  void pg_init(Real* psi, int nb) {
    pb();
    hipLaunchKernelGGL(k_pg_init<Real>, dim3(blocks_for(c.amps * nb)), dim3(256), 0, st, (V<Real>*)psi,
                       (long long)c.amps, nb);
    pe(2);
    check("k_pg_init");
  }
  template <class Real>
  void pg_copy(Real* dst, const Real* src, int nb) {
    if (hipMemcpyAsync(dst, src, c.state_bytes * nb, hipMemcpyDeviceToDevice, st) != hipSuccess && err == QF_OK) {
      err = QF_ERR_DEVICE;
      msg = "hipMemcpyAsync";
    }
  }
  template <class Real>
  void pg_rot(Real* psi, int nb, int sample0, int r, const Real* cs, const Real* cpp) {
    pb();
    hipLaunchKernelGGL(k_pg_rot<Real>, dim3(nb * c.pg_blocks), dim3(kPgThreads), 0, st, (V<Real>*)psi,
                       (long long)c.amps, c.S.runs[r].q, c.S.runs[r].coef, sample0, cs, cpp, c.S.n_coef_ps,
                       c.pg_blocks);
    pe(2);
    check("k_pg_rot");
  }
  template <class Real>
  void pg_cz(Real* psi, Real* lam, int nb, int qa, int qb) {
    pb();
    hipLaunchKernelGGL(k_pg_cz<Real>, dim3(blocks_for((c.amps >> 2) * nb)), dim3(256), 0, st, (V<Real>*)psi,
                       (V<Real>*)lam, (long long)c.amps, qa, qb, nb);
    pe(2);
    check("k_pg_cz");
  }
  // observables (any Pauli strings) of stored states; strides count reals
  template <class Real>
  void pauli_expect(const Real* psi, int64_t stride, int nb, Real* partE) {
    pb();
    hipLaunchKernelGGL(k_pauli_expect<Real>, dim3(nb * c.pauli_blocks), dim3(kPgThreads), 0, st,
                       (const V<Real>*)psi, (long long)(stride / 2), (long long)c.amps, c.C.K, d.p.pauli, partE,
                       c.pauli_blocks);
    pe(2);
    check("k_pauli_expect");
  }
  template <class Real>
  void pauli_reduce_E(int nb, int sample0, const Real* partE, Real* E) {
    const ReduceEArgsT<Real> a = make_reduce_E_args<Real>(c, nb, sample0, c.pauli_blocks, partE, E);
    pb();
    hipLaunchKernelGGL(k_reduce_E<Real>, dim3(blocks_for((long long)nb * c.C.K)), dim3(kSmallThreads), 0, st, a);
    pe(2);
    check("k_reduce_E");
  }
  template <class Real>
  void pauli_seed(const Real* psi, int64_t psi_stride, Real* lam, int64_t lam_stride, int nb, int sample0,
                  const Real* dE) {
    pb();
    hipLaunchKernelGGL(k_pauli_seed<Real>, dim3(blocks_for(c.amps * nb)), dim3(256), 0, st, (const V<Real>*)psi,
                       (long long)(psi_stride / 2), (V<Real>*)lam, (long long)(lam_stride / 2), (long long)c.amps, nb,
                       sample0, c.C.K, d.p.pauli, dE);
    pe(2);
    check("k_pauli_seed");
  }
  template <class Real>
  void pg_rot_bwd(Real* psi, Real* lam, int nb, int sample0, int r, int slot, const Real* cs, const Real* cpp,
                  Real* partF) {
    pb();
    hipLaunchKernelGGL(k_pg_rot_bwd<Real>, dim3(nb * c.pg_blocks), dim3(kPgThreads), 0, st, (V<Real>*)psi,
                       (V<Real>*)lam, (long long)c.amps, c.S.runs[r].q, c.S.runs[r].coef, sample0, cs, cpp,
                       c.S.n_coef_ps, c.pg_blocks, c.pg_chunk, slot, partF);
    pe(2);
    check("k_pg_rot_bwd");
  }
  template <class Real>
  void pg_assemble(int r0, int cnt, int nb, int sample0, const Real* th, const Real* xx, const Real* partF,
                   Real* Gr) {
    pb();
    hipLaunchKernelGGL(k_pg_assemble<Real>, dim3(blocks_for((long long)cnt * nb, 128)), dim3(128), 0, st, d.p.tabs,
                       r0, cnt, nb, c.pg_chunk, c.pg_blocks, c.n_angle, th, xx, c.C.F, sample0, partF, Gr);
    pe(2);
    check("k_pg_assemble");
  }
  template <class Real>
  void pg_reduce_grads(int nb, int sample0, const Real* Gr, Real* dtheta, Real* dx, bool accumulate) {
    const ReduceGArgsT<Real> a = make_reduce_grads_args<Real>(c, d.p, nb, sample0, Gr, dtheta, dx, accumulate);
    if (a.P == 0 && a.dx_items() == 0) return;
    pb();
    hipLaunchKernelGGL(k_reduce_grads<Real>, dim3((unsigned)reduce_grads_blocks(a)), dim3(kSmallThreads), 0, st, a);
    pe(2);
    check("k_reduce_grads");
  }
};

}  // namespace qf

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
using namespace qf;

// Workspace of qf_forward_noalloc.  Every GPU the library runs on holds its own
// copy of this array from module load until the process ends.  In host code the
// name stands for a host-side shadow, not a device address: the device address is
// taken once per device with hipGetSymbolAddress and only that pointer is used.
static __device__ __align__(256) unsigned char scratch[QF_NOALLOC_SCRATCH_BYTES];

namespace {
thread_local std::string g_last_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call
// per device, with that device current).
bool noalloc_scratch(void** out, std::string* msg) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *msg = "qf_forward_noalloc: no usable current HIP device";
    return false;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *msg = std::string("qf_forward_noalloc: hipGetSymbolAddress of the scratch array failed: ") +
             hipGetErrorString(e);
      return false;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return true;
}

qf_status fail(qf_status s, const std::string& m) {
  g_last_error = m;
  return s;
}
}  // namespace

qf_status qf::set_error(qf_status s, const std::string& m) { return fail(s, m); }

extern "C" {

const char* qf_status_string(qf_status s) {
  switch (s) {
    case QF_OK: return "ok";
    case QF_ERR_INVALID_ARG: return "invalid argument";
    case QF_ERR_UNSUPPORTED: return "unsupported";
    case QF_ERR_WORKSPACE: return "workspace too small";
    case QF_ERR_OOM: return "out of memory";
    case QF_ERR_DEVICE: return "device error";
    case QF_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* qf_last_error(void) { return g_last_error.c_str(); }

qf_status qf_circuit_create(const qf_circuit_desc* desc, qf_circuit** out) {
  if (!out) return fail(QF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::string msg;
  qf_status st = validate_circuit(desc, &msg);
  if (st != QF_OK) return fail(st, msg);
  try {
    qf_circuit* c = new qf_circuit;
    circuit_from_desc(desc, &c->c);
    *out = c;
  } catch (...) {
    return fail(QF_ERR_OOM, "host allocation failed");
  }
  return QF_OK;
}

qf_status qf_circuit_destroy(qf_circuit* c) {
  delete c;
  return QF_OK;
}

qf_status qf_plan_create(const qf_circuit* circuit, int32_t batch, const qf_tuning* tuning, qf_plan** out) {
  if (!out) return fail(QF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!circuit) return fail(QF_ERR_INVALID_ARG, "circuit is NULL");
  if (batch < 1) return fail(QF_ERR_INVALID_ARG, "batch must be >= 1");
  Tuning T;
  if (tuning) {
    T.mode = tuning->mode;
    T.k = tuning->tile_qubits;
    T.R = tuning->reg_qubits;
    T.fusion = tuning->fusion_depth;
    T.ckpt = tuning->ckpt_interval;
    T.micro = tuning->micro_batch;
    T.store = tuning->store_ckpt;
    T.memsave = tuning->mem_save;
    T.fill = tuning->epoch_fill;
    T.uncompute = tuning->uncompute;
    if (T.mode < 0 || T.mode > 2) return fail(QF_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
    if (T.k < 0 || T.k > kMaxTileQubits) return fail(QF_ERR_INVALID_ARG, "tile_qubits out of range");
    if (T.R < 0 || T.R > kMaxR) return fail(QF_ERR_INVALID_ARG, "reg_qubits out of range");
    if (T.fusion < 0 || T.ckpt < 0 || T.micro < 0) return fail(QF_ERR_INVALID_ARG, "negative tuning value");
    if (T.memsave != 0 && T.memsave != 1) return fail(QF_ERR_INVALID_ARG, "mem_save must be 0 or 1");
    if (T.memsave && T.mode != 0) return fail(QF_ERR_INVALID_ARG, "mem_save applies to the fused mode only");
    if (T.fill < -1 || T.fill > kMaxR) return fail(QF_ERR_INVALID_ARG, "epoch_fill must be -1..5");
    if (T.uncompute != 0 && T.uncompute != 1) return fail(QF_ERR_INVALID_ARG, "uncompute must be 0 or 1");
    if (T.uncompute && T.mode != 0) return fail(QF_ERR_INVALID_ARG, "uncompute applies to the fused mode only");
    if (T.uncompute && T.memsave)
      return fail(QF_ERR_INVALID_ARG, "uncompute stores no pass outputs, so mem_save does not apply");
  }
  qf_plan* p = nullptr;
  try {
    p = new qf_plan;
  } catch (...) {
    return fail(QF_ERR_OOM, "host allocation failed");
  }
  std::string msg;
  qf_status st;
  try {
    st = build_plan_core(circuit->c, batch, T, &p->core, &msg);
  } catch (const std::exception& e) {
    st = QF_ERR_INTERNAL;
    msg = e.what();
  }
  if (st == QF_OK && !p->core.per_gate && !select_pass(p->core.S.R, p->core.S.NT, false)) {
    st = QF_ERR_UNSUPPORTED;
    msg = "no pass kernel for this tile shape";
  }
  if (st == QF_OK && !p->core.per_gate) {
    // LDS of a workgroup: the pass kernels' static tile plus the adjoint pass's
    // per-wave functional sums (they grow with the runs fused into one pass),
    // and the assembly kernel's per-run sums; a plan that would exceed the
    // device limit is refused here rather than failing at launch
    int dev = 0, lim = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lim <= 0)
      lim = 64 << 10;
    const PlanCore& c = p->core;
    const size_t tile = sizeof(float2) * ((size_t)1 << c.S.R) * c.S.NT;
    const size_t need = std::max(tile + pass_shmem(c, true), assemble_shmem(c));
    if (need > (size_t)lim) {
      st = QF_ERR_UNSUPPORTED;
      msg = "a pass needs " + std::to_string(need) + " bytes of LDS per workgroup, the device allows " +
            std::to_string(lim) + ": lower fusion_depth (fewer runs per pass)";
    }
  }
  if (st == QF_OK) {
    hipGetDevice(&p->device);
    st = upload_plan(p->core, &p->dev, &msg);
  }
  if (st != QF_OK) {
    if (p->dev.blob) hipFree(p->dev.blob);
    delete p;
    return fail(st, msg);
  }
  *out = p;
  return QF_OK;
}

qf_status qf_plan_destroy(qf_plan* p) {
  if (!p) return QF_OK;
  if (p->dev.blob) hipFree(p->dev.blob);
  delete p;
  return QF_OK;
}

qf_status qf_workspace_size(const qf_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(QF_ERR_INVALID_ARG, "NULL argument");
  *bytes = p->core.ws_bytes;
  return QF_OK;
}

qf_status qf_plan_get_info(const qf_plan* p, qf_plan_info* info) {
  if (!p || !info) return fail(QF_ERR_INVALID_ARG, "NULL argument");
  const PlanCore& c = p->core;
  const Schedule& S = c.S;
  std::memset(info, 0, sizeof(*info));
  info->n_qubits = c.C.n;
  info->n_runs = (int64_t)S.runs.size();
  const double SB = (double)c.state_bytes, A = (double)c.amps;
  if (c.per_gate) {
    int64_t nrot = 0, ncz = 0;
    for (const qf_gate& g : c.C.gates) (g.kind == QF_CZ ? ncz : nrot)++;
    info->fwd_bytes_per_sample = nrot * 2 * SB + ncz * 0.5 * SB;
    info->bwd_bytes_per_sample = nrot * 4 * SB + ncz * 1.0 * SB + 2 * SB;
    info->fwd_flops_per_sample = nrot * 16 * A;
    info->bwd_flops_per_sample = nrot * 44 * A;
    info->micro_batch = c.mb;
    return QF_OK;
  }
  info->tile_qubits = S.k;
  info->reg_qubits = S.R;
  info->threads = S.NT;
  info->tiles = c.tiles;
  info->fused_passes = c.P;
  info->segments = c.n_seg;
  info->ckpt_interval = c.ckpt;
  info->micro_batch = c.mb;
  info->store_ckpt = c.store;
  info->mem_save = c.memsave;
  info->fusion_depth = S.fusion;
  info->epoch_fill = S.fill;
  info->uncompute = c.uncompute;
  info->n_perm = S.n_perm;
  info->n_u2 = S.n_u2;
  info->n_cz = S.n_cz;
  // algorithmic bytes: every forward pass reads (except the first) and writes the
  // state once; an adjoint pass reads psi and lambda and writes lambda
  const double P = c.P;
  info->fwd_bytes_per_sample = (2 * P - 1) * SB;
  // stored pass outputs of the active segment: half size in the memory-saving
  // mode, where a recompute pass writes its float32 output for the next pass
  // and a bfloat16 copy for the adjoint pass
  const double ST = c.memsave ? 0.5 * SB : SB;
  double recompute = 0, adj = 0;
  for (int s = 0; s < c.n_seg; ++s) {
    const int a = c.seg_begin[s], b = c.seg_begin[s + 1];
    if (!c.uncompute)
      for (int q = a; q <= b - 2; ++q) recompute += (q == 0 ? 0 : SB) + SB + (c.memsave ? ST : 0);
    for (int q = a; q < b; ++q)   // psi_out, lambda_out (none for the seed pass), lambda_in (none for pass 0),
                                  // psi_in in the uncompute mode (none for a segment's first pass)
      adj += (q == b - 1 ? SB : ST) + (q == c.P - 1 ? 0 : SB) + (q == 0 ? 0 : SB) +
             (c.uncompute && q > a ? SB : 0);
  }
  info->bwd_pass_bytes_per_sample = adj;
  info->bwd_bytes_per_sample = recompute + adj + (c.store ? 0 : info->fwd_bytes_per_sample);
  // algorithmic flops of a run, per amplitude, in the method's terms (one
  // fused 2x2 complex matrix per run): forward and recompute apply it (8
  // multiply-adds, 16 flops); the adjoint pass un-applies it from psi and
  // lambda and forms the gradient inner products (about 24 multiply-adds, 48
  // flops).  The kernels execute fewer: the run is a real RY between diagonal
  // phases, applied as three shears (6 flops per amplitude), so the adjoint pass
  // executes 2 x 6 + 12 (three functionals) = 24 flops per amplitude and run.
  const double runs = (double)S.n_u2;
  info->fwd_flops_per_sample = runs * 16 * A;
  double rec_runs = 0;
  for (int s = 0; s < c.n_seg && !c.uncompute; ++s)
    for (int q = c.seg_begin[s]; q <= c.seg_begin[s + 1] - 2; ++q) {
      const PassRec& pr = S.passes[q];
      rec_runs += pr.n_slots;
    }
  info->bwd_pass_flops_per_sample = runs * 48 * A;
  info->bwd_flops_per_sample = info->bwd_pass_flops_per_sample + rec_runs * 16 * A +
                               (c.store ? 0 : info->fwd_flops_per_sample);
  info->exec_bwd_pass_flops_per_sample = runs * 24 * A;
  info->bwd_pass_launches = (int64_t)c.P * ((c.B + c.mb - 1) / c.mb);
  return QF_OK;
}

static qf_status check_call(qf_plan* p, void* ws, size_t ws_bytes) {
  if (!p) return fail(QF_ERR_INVALID_ARG, "plan is NULL");
  if (!ws || ws_bytes < p->core.ws_bytes)
    return fail(QF_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, plan needs " +
                                      std::to_string(p->core.ws_bytes));
  if (((uintptr_t)ws & 255) != 0) return fail(QF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  int dev = -1;
  hipGetDevice(&dev);
  if (dev != p->device) return fail(QF_ERR_INVALID_ARG, "plan was created on another device");
  return QF_OK;
}

qf_status qf_forward_psi0(qf_plan* p, const float* theta, const float* x, const float* psi0, float* E, void* ws,
                          size_t ws_bytes, void* stream) {
  qf_status st = check_call(p, ws, ws_bytes);
  if (st != QF_OK) return st;
  const PlanCore& c = p->core;
  if (c.c128) return fail(QF_ERR_INVALID_ARG, "complex128 plan: call qf_forward_c128");
  if (!E || (c.C.P > 0 && !theta) || (c.C.F > 0 && !x)) return fail(QF_ERR_INVALID_ARG, "NULL buffer");
  GpuExec ex(c, p->dev, (hipStream_t)stream);
  ex.prof = &p->prof;
  st = run_forward(c, ex, theta, x, E, (char*)ws, psi0);
  if (st != QF_OK) return fail(st, ex.msg);
  return QF_OK;
}

qf_status qf_forward(qf_plan* p, const float* theta, const float* x, float* E, void* ws, size_t ws_bytes,
                     void* stream) {
  return qf_forward_psi0(p, theta, x, nullptr, E, ws, ws_bytes, stream);
}

qf_status qf_forward_noalloc(qf_plan* p, const float* theta, const float* x, float* E, void* stream) {
  if (!p) return fail(QF_ERR_INVALID_ARG, "plan is NULL");
  if (p->core.ws_bytes > QF_NOALLOC_SCRATCH_BYTES)
    return fail(QF_ERR_WORKSPACE, "qf_forward_noalloc: the plan needs a workspace of " +
                                      std::to_string(p->core.ws_bytes) + " bytes, more than the " +
                                      std::to_string((size_t)QF_NOALLOC_SCRATCH_BYTES) +
                                      "-byte library array; use qf_forward with a caller workspace");
  void* ws = nullptr;
  std::string msg;
  if (!noalloc_scratch(&ws, &msg)) return fail(QF_ERR_DEVICE, msg);
  qf_status st = check_call(p, ws, QF_NOALLOC_SCRATCH_BYTES);
  if (st != QF_OK) return st;
  const PlanCore& c = p->core;
  if (c.c128) return fail(QF_ERR_INVALID_ARG, "complex128 plan: call qf_forward_c128");
  if (!E || (c.C.P > 0 && !theta) || (c.C.F > 0 && !x)) return fail(QF_ERR_INVALID_ARG, "NULL buffer");
  // no profiling events on this path: it creates nothing
  GpuExec ex(c, p->dev, (hipStream_t)stream);
  st = run_forward(c, ex, theta, x, E, (char*)ws, nullptr);
  if (st != QF_OK) return fail(st, ex.msg);
  return QF_OK;
}

qf_status qf_backward_psi0(qf_plan* p, const float* theta, const float* x, const float* psi0, const float* dE,
                           float* dtheta, float* dx, void* ws, size_t ws_bytes, void* stream) {
  qf_status st = check_call(p, ws, ws_bytes);
  if (st != QF_OK) return st;
  const PlanCore& c = p->core;
  if (c.c128) return fail(QF_ERR_INVALID_ARG, "complex128 plan: call qf_backward_c128");
  if (!dE || (c.C.P > 0 && (!theta || !dtheta)) || (c.C.F > 0 && !x))
    return fail(QF_ERR_INVALID_ARG, "NULL buffer");
  GpuExec ex(c, p->dev, (hipStream_t)stream);
  ex.prof = &p->prof;
  ex.theta = theta;
  ex.x = x;
  ex.cp = coef_ptrs(c, (char*)ws);
  st = run_backward(c, ex, theta, x, dE, dtheta, dx, (char*)ws, psi0);
  if (st != QF_OK) return fail(st, ex.msg);
  return QF_OK;
}

qf_status qf_backward(qf_plan* p, const float* theta, const float* x, const float* dE, float* dtheta, float* dx,
                      void* ws, size_t ws_bytes, void* stream) {
  return qf_backward_psi0(p, theta, x, nullptr, dE, dtheta, dx, ws, ws_bytes, stream);
}

qf_status qf_forward_c128(qf_plan* p, const double* theta, const double* x, const double* psi0, double* E,
                          void* ws, size_t ws_bytes, void* stream) {
  qf_status st = check_call(p, ws, ws_bytes);
  if (st != QF_OK) return st;
  const PlanCore& c = p->core;
  if (!c.c128) return fail(QF_ERR_INVALID_ARG, "plan is not a complex128 plan (tuning mode 2)");
  if (!E || (c.C.P > 0 && !theta) || (c.C.F > 0 && !x)) return fail(QF_ERR_INVALID_ARG, "NULL buffer");
  GpuExec ex(c, p->dev, (hipStream_t)stream);
  ex.prof = &p->prof;
  st = run_forward_pg<double>(c, ex, theta, x, E, (char*)ws, psi0);
  if (st != QF_OK) return fail(st, ex.msg);
  return QF_OK;
}

qf_status qf_backward_c128(qf_plan* p, const double* theta, const double* x, const double* dE, double* dtheta,
                           double* dx, void* ws, size_t ws_bytes, void* stream) {
  qf_status st = check_call(p, ws, ws_bytes);
  if (st != QF_OK) return st;
  const PlanCore& c = p->core;
  if (!c.c128) return fail(QF_ERR_INVALID_ARG, "plan is not a complex128 plan (tuning mode 2)");
  if (!dE || (c.C.P > 0 && (!theta || !dtheta)) || (c.C.F > 0 && !x))
    return fail(QF_ERR_INVALID_ARG, "NULL buffer");
  GpuExec ex(c, p->dev, (hipStream_t)stream);
  ex.prof = &p->prof;
  st = run_backward_pg<double>(c, ex, theta, x, dE, dtheta, dx, (char*)ws);
  if (st != QF_OK) return fail(st, ex.msg);
  return QF_OK;
}

qf_status qf_profile_enable(qf_plan* p, int enable) {
  if (!p) return fail(QF_ERR_INVALID_ARG, "plan is NULL");
  p->prof.on = enable != 0;
  p->prof.used = 0;
  return QF_OK;
}

qf_status qf_profile_read(qf_plan* p, qf_profile* out) {
  if (!p || !out) return fail(QF_ERR_INVALID_ARG, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  Profiler& pr = p->prof;
  for (size_t i = 0; i < pr.used; ++i) {
    hipEvent_t a = pr.ev[2 * i], b = pr.ev[2 * i + 1];
    if (hipEventSynchronize(b) != hipSuccess) return fail(QF_ERR_DEVICE, "hipEventSynchronize failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return fail(QF_ERR_DEVICE, "hipEventElapsedTime failed");
    const int k = pr.kind[i];
    out->launches[k] += 1;
    out->ms[k] += ms;
  }
  pr.used = 0;
  return QF_OK;
}

}  // extern "C"
