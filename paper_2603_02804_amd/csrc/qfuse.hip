// qfuse.hip -- gfx950 kernels, their launch backend and the C-ABI (include/qfuse.h).
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
//   k_reduce_E          expectation partial sums -> E[b][k] (App. B.2, Z strings).
//   k_pg_*              one-kernel-per-gate baseline.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "driver.hpp"

namespace qf {

// ---------------------------------------------------------------------------
// pass kernel
// ---------------------------------------------------------------------------
struct KArgs {
  const Op* ops;
  const LayoutRec* layouts;
  const CzGroup* czg;
  const FuncEntry* funcs;
  const PassRec* prec;
  const float* coef_sh;
  const float* coef_ps;
  const float2* src0;
  const float2* src1;
  float2* dst;
  float* partF;
  float* partE;
  const float* dE;
  const uint32_t* zmask;
  long long s0, s1, sd;       // per-sample strides (float2 units)
  int n_ops;
  int n_ps;
  int K;
  int sample0;
  int tiles_log2;
  int tb;                     // thread bits of the tile
  int do_expect;
};

// Register-bit dispatch: expands STMT(J) for the compile-time bit J == j.
#define QF_WITH_BIT(R, j, STMT)                      \
  switch (j) {                                       \
    case 0: { constexpr int J = 0; STMT; } break;    \
    case 1: if constexpr (R > 1) { constexpr int J = 1; STMT; } break; \
    case 2: if constexpr (R > 2) { constexpr int J = 2; STMT; } break; \
    case 3: if constexpr (R > 3) { constexpr int J = 3; STMT; } break; \
    case 4: if constexpr (R > 4) { constexpr int J = 4; STMT; } break; \
    default: break;                                  \
  }

__device__ __forceinline__ uint32_t tbase(const uint32_t* __restrict__ tab, int t, int tb) {
  uint32_t v = 0;
#pragma unroll
  for (int i = 0; i < kMaxThreadBits; ++i)
    if (i < tb && ((t >> i) & 1)) v ^= tab[i];
  return v;
}

struct U2c {
  float r00, i00, r01, i01, r10, i10, r11, i11;
};

template <int R, int J>
__device__ __forceinline__ void apply_u2(float2 (&a)[1 << R], const U2c& u) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    constexpr int s = 1 << J;
    const float2 x0 = a[i], x1 = a[i | s];
    float2 y0, y1;
    y0.x = u.r00 * x0.x - u.i00 * x0.y + u.r01 * x1.x - u.i01 * x1.y;
    y0.y = u.r00 * x0.y + u.i00 * x0.x + u.r01 * x1.y + u.i01 * x1.x;
    y1.x = u.r10 * x0.x - u.i10 * x0.y + u.r11 * x1.x - u.i11 * x1.y;
    y1.y = u.r10 * x0.y + u.i10 * x0.x + u.r11 * x1.y + u.i11 * x1.x;
    a[i] = y0;
    a[i | s] = y1;
  }
}

// Im<l|X_q|a>, Im<l|Y_q|a>, Im<l|Z_q|a> over the pairs along register bit J.
template <int R, int J>
__device__ __forceinline__ void func3(const float2 (&a)[1 << R], const float2 (&l)[1 << R], float& fx, float& fy,
                                      float& fz) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    constexpr int s = 1 << J;
    const float2 p0 = a[i], p1 = a[i | s], l0 = l[i], l1 = l[i | s];
    fx += l0.x * p1.y - l0.y * p1.x + l1.x * p0.y - l1.y * p0.x;
    fy += (l1.x * p0.x + l1.y * p0.y) - (l0.x * p1.x + l0.y * p1.y);
    fz += (l0.x * p0.y - l0.y * p0.x) - (l1.x * p1.y - l1.y * p1.x);
  }
}

// Butterfly reduce-scatter of 16 per-lane values over a wave of 64 lanes.
// Afterwards lane L holds the wave sum of value ((L >> 2) & 15).
__device__ __forceinline__ float wave_reduce16(float (&v)[16], int lane) {
  {
    const bool hi = (lane & 32) != 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float send = hi ? v[i] : v[i + 8];
      const float keep = hi ? v[i + 8] : v[i];
      v[i] = keep + __shfl_xor(send, 32);
    }
  }
  {
    const bool hi = (lane & 16) != 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float send = hi ? v[i] : v[i + 4];
      const float keep = hi ? v[i + 4] : v[i];
      v[i] = keep + __shfl_xor(send, 16);
    }
  }
  {
    const bool hi = (lane & 8) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float send = hi ? v[i] : v[i + 2];
      const float keep = hi ? v[i + 2] : v[i];
      v[i] = keep + __shfl_xor(send, 8);
    }
  }
  {
    const bool hi = (lane & 4) != 0;
    const float send = hi ? v[0] : v[1];
    const float keep = hi ? v[1] : v[0];
    v[0] = keep + __shfl_xor(send, 4);
  }
  v[0] += __shfl_xor(v[0], 2);
  v[0] += __shfl_xor(v[0], 1);
  return v[0];
}

__device__ __forceinline__ U2c load_u2(const KArgs& A, int ref, int sample, bool adjoint) {
  const float* p = ref >= 0 ? A.coef_sh + 8 * (size_t)ref : A.coef_ps + 8 * ((size_t)sample * A.n_ps + (-1 - ref));
  U2c u;
  if (!adjoint) {
    u.r00 = p[0]; u.i00 = p[1]; u.r01 = p[2]; u.i01 = p[3];
    u.r10 = p[4]; u.i10 = p[5]; u.r11 = p[6]; u.i11 = p[7];
  } else {   // u^dagger
    u.r00 = p[0]; u.i00 = -p[1]; u.r01 = p[4]; u.i01 = -p[5];
    u.r10 = p[2]; u.i10 = -p[3]; u.r11 = p[6]; u.i11 = -p[7];
  }
  return u;
}

template <int R, int NT, bool BWD>
__global__ __launch_bounds__(NT) void k_pass(const KArgs A) {
  extern __shared__ float2 lds[];
  constexpr int NA = 1 << R;
  constexpr int WAVES = NT / 64;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int tb = A.tb;
  const bool active = t < (1 << tb);
  const int item = blockIdx.x;
  const int sl = item >> A.tiles_log2;
  const int tile = item & ((1 << A.tiles_log2) - 1);
  const int sample = A.sample0 + sl;
  const PassRec* __restrict__ P = A.prec;

  uint32_t tlog = 0, tin = 0, tout = 0;
  for (int i = 0; i < P->n_nonlocal; ++i)
    if ((tile >> i) & 1) {
      tlog |= 1u << P->nl_log[i];
      tin |= 1u << P->nl_in[i];
      tout |= 1u << P->nl_out[i];
    }

  float2 a[NA];
  float2 l[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    a[j] = make_float2(0.f, 0.f);
    l[j] = make_float2(0.f, 0.f);
  }
  const int n_slots = P->n_slots;

  for (int oi = 0; oi < A.n_ops; ++oi) {
    const Op op = A.ops[oi];
    switch (op.kind) {
      case OP_INIT0: {
        const LayoutRec* __restrict__ L = A.layouts + op.a;
        const uint32_t base = tlog | tbase(L->log_thr, t, tb);
#pragma unroll
        for (int jj = 0; jj < NA; ++jj)
          a[jj] = make_float2((active && (base | L->log_reg[jj]) == 0u) ? 1.f : 0.f, 0.f);
        break;
      }
      case OP_LOAD: {
        const LayoutRec* __restrict__ L = A.layouts + op.a;
        const uint32_t base = (op.c ? tout : tin) | tbase(L->mem_thr, t, tb);
        if (active) {
          if (op.b == 0) {
            const float2* __restrict__ src = A.src0 + (long long)sl * A.s0;
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) a[jj] = src[base | L->mem_reg[jj]];
          } else if constexpr (BWD) {
            const float2* __restrict__ src = A.src1 + (long long)sl * A.s1;
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) l[jj] = src[base | L->mem_reg[jj]];
          }
        }
        break;
      }
      case OP_STORE: {
        const LayoutRec* __restrict__ L = A.layouts + op.a;
        const uint32_t base = (op.c ? tout : tin) | tbase(L->mem_thr, t, tb);
        if (active && A.dst) {
          float2* __restrict__ dst = A.dst + (long long)sl * A.sd;
          if constexpr (BWD) {
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) dst[base | L->mem_reg[jj]] = l[jj];
          } else {
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) dst[base | L->mem_reg[jj]] = a[jj];
          }
        }
        break;
      }
      case OP_PERM: {
        const LayoutRec* __restrict__ F = A.layouts + op.a;
        const LayoutRec* __restrict__ T = A.layouts + op.b;
        const uint32_t bf = tbase(F->lds_thr, t, tb);
        const uint32_t bt = tbase(T->lds_thr, t, tb);
        if (active) {
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) lds[bf ^ F->lds_reg[jj]] = a[jj];
        }
        __syncthreads();
        if (active) {
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) a[jj] = lds[bt ^ T->lds_reg[jj]];
        }
        __syncthreads();
        if constexpr (BWD) {
          if (active) {
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) lds[bf ^ F->lds_reg[jj]] = l[jj];
          }
          __syncthreads();
          if (active) {
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) l[jj] = lds[bt ^ T->lds_reg[jj]];
          }
          __syncthreads();
        }
        break;
      }
      case OP_U2: {
        const U2c u = load_u2(A, op.b, sample, false);
        QF_WITH_BIT(R, op.a, (apply_u2<R, J>(a, u)));
        break;
      }
      case OP_U2ADJ: {
        if constexpr (BWD) {
          const U2c u = load_u2(A, op.b, sample, true);
          QF_WITH_BIT(R, op.a, (apply_u2<R, J>(a, u), apply_u2<R, J>(l, u)));
        }
        break;
      }
      case OP_CZ: {
        const LayoutRec* __restrict__ L = A.layouts + op.a;
        const uint32_t base = tlog | tbase(L->log_thr, t, tb);
        const CzGroup* __restrict__ g = A.czg + op.b;
        const int ng = op.c;
#pragma unroll
        for (int jj = 0; jj < NA; ++jj) {
          const uint32_t x = base | L->log_reg[jj];
          uint32_t par = 0;
          for (int i = 0; i < ng; ++i) par ^= x & (x >> g[i].shift) & g[i].mask;
          const uint32_t flip = (uint32_t)(__popc(par) & 1) << 31;
          a[jj].x = __uint_as_float(__float_as_uint(a[jj].x) ^ flip);
          a[jj].y = __uint_as_float(__float_as_uint(a[jj].y) ^ flip);
          if constexpr (BWD) {
            l[jj].x = __uint_as_float(__float_as_uint(l[jj].x) ^ flip);
            l[jj].y = __uint_as_float(__float_as_uint(l[jj].y) ^ flip);
          }
        }
        break;
      }
      case OP_EXPECT: {
        if constexpr (!BWD) {
          if (!A.do_expect) break;
          const LayoutRec* __restrict__ L = A.layouts + op.a;
          const uint32_t base = tlog | tbase(L->log_thr, t, tb);
          for (int k0 = 0; k0 < A.K; k0 += 16) {
            float v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = 0.f;
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) {
              const uint32_t x = base | L->log_reg[jj];
              const float p = a[jj].x * a[jj].x + a[jj].y * a[jj].y;
#pragma unroll
              for (int k = 0; k < 16; ++k)
                if (k0 + k < A.K) v[k] += (__popc(x & A.zmask[k0 + k]) & 1) ? -p : p;
            }
            const float s = wave_reduce16(v, lane);
            const int idx = (lane >> 2) & 15;
            if ((lane & 3) == 0 && k0 + idx < A.K)
              A.partE[((size_t)item * WAVES + wave) * A.K + k0 + idx] = s;
          }
        }
        break;
      }
      case OP_SEED: {
        if constexpr (BWD) {
          const LayoutRec* __restrict__ L = A.layouts + op.a;
          const uint32_t base = tlog | tbase(L->log_thr, t, tb);
          const float* __restrict__ g = A.dE + (size_t)sample * A.K;
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) {
            const uint32_t x = base | L->log_reg[jj];
            float c = 0.f;
            for (int k = 0; k < A.K; ++k) c += (__popc(x & A.zmask[k]) & 1) ? -g[k] : g[k];
            l[jj] = make_float2(2.f * c * a[jj].x, 2.f * c * a[jj].y);
          }
        }
        break;
      }
      case OP_FUNC: {
        if constexpr (BWD) {
          const FuncEntry* __restrict__ fe = A.funcs + op.b;
          const int m = op.a;
          float v[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) v[i] = 0.f;
#pragma unroll
          for (int e = 0; e < R; ++e) {
            if (e < m) {
              QF_WITH_BIT(R, fe[e].regbit, (func3<R, J>(a, l, v[3 * e], v[3 * e + 1], v[3 * e + 2])));
            }
          }
          const float s = wave_reduce16(v, lane);
          const int idx = (lane >> 2) & 15;
          if ((lane & 3) == 0 && idx < 3 * m) {
            const int e = idx / 3, pq = idx - 3 * e;
            A.partF[((size_t)item * WAVES + wave) * 3 * n_slots + 3 * fe[e].slot + pq] = s;
          }
        }
        break;
      }
      default:
        break;
    }
  }
}

// ---------------------------------------------------------------------------
// small kernels: coefficients, gradient assembly, reductions
// ---------------------------------------------------------------------------
struct D2 {
  double r[4], i[4];   // row-major 2x2 complex
};

__device__ inline D2 d2_mul(const D2& a, const D2& b) {
  D2 c;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      double re = 0, im = 0;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        re += a.r[2 * r + k] * b.r[2 * k + q] - a.i[2 * r + k] * b.i[2 * k + q];
        im += a.r[2 * r + k] * b.i[2 * k + q] + a.i[2 * r + k] * b.r[2 * k + q];
      }
      c.r[2 * r + q] = re;
      c.i[2 * r + q] = im;
    }
  return c;
}

__device__ inline D2 d2_eye() {
  D2 u;
  for (int i = 0; i < 4; ++i) u.r[i] = u.i[i] = 0;
  u.r[0] = u.r[3] = 1;
  return u;
}

__device__ inline D2 d2_rot(int kind, double phi) {
  double s, c;
  sincos(0.5 * phi, &s, &c);
  D2 u;
  for (int i = 0; i < 4; ++i) u.r[i] = u.i[i] = 0;
  if (kind == QF_RX) { u.r[0] = c; u.i[1] = -s; u.i[2] = -s; u.r[3] = c; }
  else if (kind == QF_RY) { u.r[0] = c; u.r[1] = -s; u.r[2] = s; u.r[3] = c; }
  else { u.r[0] = c; u.i[0] = -s; u.r[3] = c; u.i[3] = s; }
  return u;
}

__device__ inline D2 d2_pauli(int kind) {
  D2 p;
  for (int i = 0; i < 4; ++i) p.r[i] = p.i[i] = 0;
  if (kind == QF_RX) { p.r[1] = 1; p.r[2] = 1; }
  else if (kind == QF_RY) { p.i[1] = -1; p.i[2] = 1; }
  else { p.r[0] = 1; p.r[3] = -1; }
  return p;
}

__device__ inline D2 d2_dag(const D2& a) {
  D2 d;
  d.r[0] = a.r[0]; d.i[0] = -a.i[0];
  d.r[1] = a.r[2]; d.i[1] = -a.i[2];
  d.r[2] = a.r[1]; d.i[2] = -a.i[1];
  d.r[3] = a.r[3]; d.i[3] = -a.i[3];
  return d;
}

struct Tabs {
  const RunRec* runs;
  const int32_t* run_gates;
  const GateRec* gates;
  const int32_t* coef_runs_sh;
  const int32_t* coef_runs_ps;
  const PassRec* passes;
  const int64_t* partF_off;
  const int32_t* seg_runs;
  const int32_t* seg_run_begin;
  const int32_t* th_ref_begin;
  const int32_t* th_refs;
  const int32_t* in_ref_begin;
  const int32_t* in_refs;
};

__device__ inline double gate_angle(const GateRec& g, const float* theta, const float* x, int F, int sample) {
  return g.theta_idx >= 0 ? (double)theta[g.theta_idx] : (double)x[(size_t)sample * F + g.input_idx];
}

__global__ void k_coef(Tabs T, const float* theta, const float* x, int F, int n_sh, int n_ps, int B, float* csh,
                       float* cps) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = n_sh + (long long)n_ps * B;
  if (idx >= total) return;
  int r, sample;
  float* out;
  if (idx < n_sh) {
    r = T.coef_runs_sh[idx];
    sample = 0;
    out = csh + 8 * idx;
  } else {
    const long long j = idx - n_sh;
    sample = (int)(j / n_ps);
    const int i = (int)(j - (long long)sample * n_ps);
    r = T.coef_runs_ps[i];
    out = cps + 8 * j;
  }
  const RunRec rr = T.runs[r];
  D2 U = d2_eye();
  for (int i = 0; i < rr.gate_count; ++i) {
    const GateRec g = T.gates[T.run_gates[rr.gate_begin + i]];
    U = d2_mul(d2_rot(g.kind, gate_angle(g, theta, x, F, sample)), U);
  }
  for (int i = 0; i < 4; ++i) {
    out[2 * i] = (float)U.r[i];
    out[2 * i + 1] = (float)U.i[i];
  }
}

__device__ inline void run_grads(const Tabs& T, int r, const float* theta, const float* x, int F, int sample,
                                 double fx, double fy, double fz, float* Grow) {
  const RunRec rr = T.runs[r];
  D2 K = d2_eye();
  for (int i = rr.gate_count - 1; i >= 0; --i) {
    const GateRec g = T.gates[T.run_gates[rr.gate_begin + i]];
    const D2 G = d2_mul(d2_mul(K, d2_pauli(g.kind)), d2_dag(K));
    Grow[g.out_idx] = (float)(0.5 * (G.r[2] * fx + G.i[2] * fy + G.r[0] * fz));
    K = d2_mul(K, d2_rot(g.kind, gate_angle(g, theta, x, F, sample)));
  }
}

__global__ void k_assemble(Tabs T, int seg, int nb, int sample0, int tiles_waves, int n_angle, const float* theta,
                           const float* x, int F, const float* partF, float* Gr) {
  const int r0 = T.seg_run_begin[seg], nr = T.seg_run_begin[seg + 1] - r0;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nr * nb) return;
  const int s = (int)(idx / nr), i = (int)(idx - (long long)s * nr);
  const int r = T.seg_runs[r0 + i];
  const RunRec rr = T.runs[r];
  const int ns = T.passes[rr.pass].n_slots;
  const float* base = partF + (long long)nb * T.partF_off[rr.pass] + (long long)s * tiles_waves * 3 * ns + 3 * rr.slot;
  double f0 = 0, f1 = 0, f2 = 0;
  for (int it = 0; it < tiles_waves; ++it) {
    const float* p = base + (long long)it * 3 * ns;
    f0 += p[0];
    f1 += p[1];
    f2 += p[2];
  }
  run_grads(T, r, theta, x, F, sample0 + s, f0, f1, f2, Gr + (long long)s * n_angle);
}

__global__ void k_reduce_grads(Tabs T, int nb, int sample0, int n_angle, int P, int F, const float* Gr,
                               float* dtheta, float* dx, int accumulate) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < P) {
    const int p = (int)idx;
    double acc = 0;
    for (int s = 0; s < nb; ++s)
      for (int i = T.th_ref_begin[p]; i < T.th_ref_begin[p + 1]; ++i) acc += Gr[(long long)s * n_angle + T.th_refs[i]];
    dtheta[p] = accumulate ? dtheta[p] + (float)acc : (float)acc;
  } else if (dx && idx < P + (long long)nb * F) {
    const long long j = idx - P;
    const int s = (int)(j / F), f = (int)(j - (long long)s * F);
    double acc = 0;
    for (int i = T.in_ref_begin[f]; i < T.in_ref_begin[f + 1]; ++i) acc += Gr[(long long)s * n_angle + T.in_refs[i]];
    dx[(long long)(sample0 + s) * F + f] = (float)acc;
  }
}

__global__ void k_reduce_E(int nb, int sample0, int parts, int K, const float* partE, float* E) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * K) return;
  const int s = idx / K, k = idx - s * K;
  double acc = 0;
  for (int i = 0; i < parts; ++i) acc += partE[((long long)s * parts + i) * K + k];
  E[(long long)(sample0 + s) * K + k] = (float)acc;
}

// ---------------------------------------------------------------------------
// per-gate baseline kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long pair_lo(long long p, int q) {
  return ((p >> q) << (q + 1)) | (p & ((1ll << q) - 1));
}

__global__ void k_pg_init(float2* psi, long long amps, int nb) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= amps * nb) return;
  psi[i] = make_float2((i % amps) == 0 ? 1.f : 0.f, 0.f);
}

__global__ __launch_bounds__(kPgThreads) void k_pg_rot(float2* psi, long long amps, int q, int ref, int sample0,
                                                       const float* csh, const float* cps, int n_ps, int blocks) {
  const int s = blockIdx.x / blocks, blk = blockIdx.x - s * blocks;
  float2* v = psi + (long long)s * amps;
  const float* c = ref >= 0 ? csh + 8 * (long long)ref : cps + 8 * ((long long)(sample0 + s) * n_ps + (-1 - ref));
  const float r00 = c[0], i00 = c[1], r01 = c[2], i01 = c[3], r10 = c[4], i10 = c[5], r11 = c[6], i11 = c[7];
  const long long pairs = amps >> 1;
#pragma unroll
  for (int k = 0; k < kPgPairsPerThread; ++k) {
    const long long p = ((long long)blk * kPgPairsPerThread + k) * kPgThreads + threadIdx.x;
    if (p >= pairs) break;
    const long long i0 = pair_lo(p, q), i1 = i0 | (1ll << q);
    const float2 x0 = v[i0], x1 = v[i1];
    v[i0] = make_float2(r00 * x0.x - i00 * x0.y + r01 * x1.x - i01 * x1.y, r00 * x0.y + i00 * x0.x + r01 * x1.y + i01 * x1.x);
    v[i1] = make_float2(r10 * x0.x - i10 * x0.y + r11 * x1.x - i11 * x1.y, r10 * x0.y + i10 * x0.x + r11 * x1.y + i11 * x1.x);
  }
}

// CZ touches only the quarter of the amplitudes with both bits set.
__global__ void k_pg_cz(float2* psi, float2* lam, long long amps, int qa, int qb, int nb) {
  const long long quarter = amps >> 2;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= quarter * nb) return;
  const long long s = idx / quarter, j = idx - s * quarter;
  const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
  long long i = pair_lo(j, lo);
  i = pair_lo(i, hi);
  i |= (1ll << lo) | (1ll << hi);
  float2* v = psi + s * amps + i;
  *v = make_float2(-v->x, -v->y);
  if (lam) {
    float2* w = lam + s * amps + i;
    *w = make_float2(-w->x, -w->y);
  }
}

// Block sum of NV per-thread values; writes the first `count` sums to out[0..count).
template <int NV>
__device__ inline void block_reduce(float (&v)[NV], float* out, int count) {
  __shared__ float sm[NV][kPgThreads / 64];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    float x = v[k];
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
    if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < NV && (int)threadIdx.x < count) {
    float acc = 0;
    for (int w = 0; w < kPgThreads / 64; ++w) acc += sm[threadIdx.x][w];
    out[threadIdx.x] = acc;
  }
}

__global__ __launch_bounds__(kPgThreads) void k_pg_expect(const float2* psi, long long amps, int K,
                                                          const uint32_t* zmask, float* partE, int blocks) {
  const int s = blockIdx.x / blocks, blk = blockIdx.x - s * blocks;
  const float2* v = psi + (long long)s * amps;
  for (int k0 = 0; k0 < K; k0 += 8) {
    float acc[8];
    for (int k = 0; k < 8; ++k) acc[k] = 0;
    for (int k2 = 0; k2 < 2 * kPgPairsPerThread; ++k2) {
      const long long i = ((long long)blk * 2 * kPgPairsPerThread + k2) * kPgThreads + threadIdx.x;
      if (i >= amps) break;
      const float p = v[i].x * v[i].x + v[i].y * v[i].y;
      for (int k = 0; k < 8; ++k)
        if (k0 + k < K) acc[k] += (__popcll((unsigned long long)i & zmask[k0 + k]) & 1) ? -p : p;
    }
    block_reduce<8>(acc, partE + ((long long)s * blocks + blk) * K + k0, K - k0);
    __syncthreads();
  }
}

__global__ void k_pg_seed(const float2* psi, float2* lam, long long amps, int nb, int sample0, int K,
                          const uint32_t* zmask, const float* dE) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= amps * nb) return;
  const long long s = idx / amps, i = idx - s * amps;
  float c = 0;
  for (int k = 0; k < K; ++k) {
    const float g = dE[(sample0 + s) * K + k];
    c += (__popcll((unsigned long long)i & zmask[k]) & 1) ? -g : g;
  }
  lam[idx] = make_float2(2.f * c * psi[idx].x, 2.f * c * psi[idx].y);
}

__global__ __launch_bounds__(kPgThreads) void k_pg_rot_bwd(float2* psi, float2* lam, long long amps, int q, int ref,
                                                           int sample0, const float* csh, const float* cps, int n_ps,
                                                           int blocks, int chunk, int slot, float* partF) {
  const int s = blockIdx.x / blocks, blk = blockIdx.x - s * blocks;
  float2* v = psi + (long long)s * amps;
  float2* w = lam + (long long)s * amps;
  const float* c = ref >= 0 ? csh + 8 * (long long)ref : cps + 8 * ((long long)(sample0 + s) * n_ps + (-1 - ref));
  // u^dagger
  const float r00 = c[0], i00 = -c[1], r01 = c[4], i01 = -c[5], r10 = c[2], i10 = -c[3], r11 = c[6], i11 = -c[7];
  const long long pairs = amps >> 1;
  float f[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < kPgPairsPerThread; ++k) {
    const long long p = ((long long)blk * kPgPairsPerThread + k) * kPgThreads + threadIdx.x;
    if (p >= pairs) break;
    const long long i0 = pair_lo(p, q), i1 = i0 | (1ll << q);
    const float2 p0 = v[i0], p1 = v[i1], l0 = w[i0], l1 = w[i1];
    f[0] += l0.x * p1.y - l0.y * p1.x + l1.x * p0.y - l1.y * p0.x;
    f[1] += (l1.x * p0.x + l1.y * p0.y) - (l0.x * p1.x + l0.y * p1.y);
    f[2] += (l0.x * p0.y - l0.y * p0.x) - (l1.x * p1.y - l1.y * p1.x);
    v[i0] = make_float2(r00 * p0.x - i00 * p0.y + r01 * p1.x - i01 * p1.y, r00 * p0.y + i00 * p0.x + r01 * p1.y + i01 * p1.x);
    v[i1] = make_float2(r10 * p0.x - i10 * p0.y + r11 * p1.x - i11 * p1.y, r10 * p0.y + i10 * p0.x + r11 * p1.y + i11 * p1.x);
    w[i0] = make_float2(r00 * l0.x - i00 * l0.y + r01 * l1.x - i01 * l1.y, r00 * l0.y + i00 * l0.x + r01 * l1.y + i01 * l1.x);
    w[i1] = make_float2(r10 * l0.x - i10 * l0.y + r11 * l1.x - i11 * l1.y, r10 * l0.y + i10 * l0.x + r11 * l1.y + i11 * l1.x);
  }
  block_reduce<3>(f, partF + (((long long)s * chunk + slot) * blocks + blk) * 3, 3);
}

__global__ void k_pg_assemble(Tabs T, int r0, int cnt, int nb, int chunk, int blocks, int n_angle,
                              const float* theta, const float* x, int F, int sample0, const float* partF, float* Gr) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)cnt * nb) return;
  const int s = (int)(idx / cnt), i = (int)(idx - (long long)s * cnt);
  const int r = r0 + i, slot = r % chunk;
  double f[3] = {0, 0, 0};
  for (int b = 0; b < blocks; ++b)
    for (int P = 0; P < 3; ++P) f[P] += partF[(((long long)s * chunk + slot) * blocks + b) * 3 + P];
  run_grads(T, r, theta, x, F, sample0 + s, f[0], f[1], f[2], Gr + (long long)s * n_angle);
}

// ---------------------------------------------------------------------------
// device plan and launch backend
// ---------------------------------------------------------------------------
struct DevPlan {
  char* blob = nullptr;
  size_t bytes = 0;
  const Op* ops = nullptr;
  const LayoutRec* layouts = nullptr;
  const CzGroup* czg = nullptr;
  const FuncEntry* funcs = nullptr;
  const PassRec* passes = nullptr;
  const uint32_t* zmask = nullptr;
  Tabs tabs{};
};

template <class T>
static void push_table(std::vector<char>& blob, std::vector<size_t>& offs, const std::vector<T>& v) {
  size_t off = align_up(blob.size());
  blob.resize(off + std::max<size_t>(sizeof(T), v.size() * sizeof(T)), 0);
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
  offs.push_back(off);
}

static qf_status upload_plan(const PlanCore& c, DevPlan* d, std::string* msg) {
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
  d->ops = (const Op*)(b + o[0]);
  d->layouts = (const LayoutRec*)(b + o[1]);
  d->czg = (const CzGroup*)(b + o[2]);
  d->funcs = (const FuncEntry*)(b + o[3]);
  d->passes = (const PassRec*)(b + o[4]);
  d->zmask = (const uint32_t*)(b + o[5]);
  Tabs& t = d->tabs;
  t.runs = (const RunRec*)(b + o[6]);
  t.run_gates = (const int32_t*)(b + o[7]);
  t.gates = (const GateRec*)(b + o[8]);
  t.coef_runs_sh = (const int32_t*)(b + o[9]);
  t.coef_runs_ps = (const int32_t*)(b + o[10]);
  t.passes = d->passes;
  t.partF_off = (const int64_t*)(b + o[11]);
  t.seg_runs = (const int32_t*)(b + o[12]);
  t.seg_run_begin = (const int32_t*)(b + o[13]);
  t.th_ref_begin = (const int32_t*)(b + o[14]);
  t.th_refs = (const int32_t*)(b + o[15]);
  t.in_ref_begin = (const int32_t*)(b + o[16]);
  t.in_refs = (const int32_t*)(b + o[17]);
  return QF_OK;
}

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
  if (NT != 64) return nullptr;
  switch (R) {
    case 1: return bwd ? pass_fn<1, 64, true>() : pass_fn<1, 64, false>();
    case 2: return bwd ? pass_fn<2, 64, true>() : pass_fn<2, 64, false>();
    case 3: return bwd ? pass_fn<3, 64, true>() : pass_fn<3, 64, false>();
    case 4: return bwd ? pass_fn<4, 64, true>() : pass_fn<4, 64, false>();
    default: return nullptr;
  }
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

struct GpuExec {
  const PlanCore& c;
  const DevPlan& d;
  hipStream_t st;
  Profiler* prof = nullptr;
  void pb() { if (prof) prof->begin(st); }
  void pe(int k) { if (prof) prof->end(st, k); }
  const float* theta = nullptr;
  const float* x = nullptr;
  const float* csh = nullptr;
  const float* cps = nullptr;
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
  static unsigned blocks_for(long long n, int t = 256) { return (unsigned)std::max<long long>(1, (n + t - 1) / t); }

  void coef(const float* th, const float* xx, float* cs, float* cp) {
    theta = th; x = xx; csh = cs; cps = cp;
    const long long total = c.S.n_coef_shared + (long long)c.S.n_coef_ps * c.B;
    if (total == 0) return;
    pb();
    hipLaunchKernelGGL(k_coef, dim3(blocks_for(total)), dim3(256), 0, st, d.tabs, th, xx, c.C.F, c.S.n_coef_shared,
                       c.S.n_coef_ps, c.B, cs, cp);
    pe(2);
    check("k_coef");
  }

  void pass(const PassLaunch& L) {
    const Schedule& S = c.S;
    const PassRec& pr = S.passes[L.pass];
    KArgs A;
    A.ops = d.ops + (L.bwd ? pr.bop_begin : pr.fop_begin);
    A.n_ops = L.bwd ? pr.bop_count : pr.fop_count;
    A.layouts = d.layouts;
    A.czg = d.czg;
    A.funcs = d.funcs;
    A.prec = d.passes + L.pass;
    A.coef_sh = csh;
    A.coef_ps = cps;
    A.n_ps = S.n_coef_ps;
    A.src0 = (const float2*)L.src0;
    A.s0 = L.src0_stride / 2;
    A.src1 = (const float2*)L.src1;
    A.s1 = L.src1_stride / 2;
    A.dst = (float2*)L.dst;
    A.sd = L.dst_stride / 2;
    A.partF = L.partF;
    A.partE = L.partE;
    A.dE = L.dE;
    A.zmask = d.zmask;
    A.K = c.C.K;
    A.sample0 = L.sample0;
    A.tiles_log2 = S.tiles_log2;
    A.tb = S.thread_bits;
    A.do_expect = L.do_expect;
    PassFn fn = select_pass(S.R, S.NT, L.bwd);
    if (!fn) {
      if (err == QF_OK) { err = QF_ERR_UNSUPPORTED; msg = "no pass kernel for this tile shape"; }
      return;
    }
    const size_t shmem = sizeof(float2) << S.k;
    pb();
    hipLaunchKernelGGL(fn, dim3((unsigned)((long long)L.nb << S.tiles_log2)), dim3(S.NT), shmem, st, A);
    pe(L.bwd ? 1 : 0);
    check(L.bwd ? "k_pass(bwd)" : "k_pass(fwd)");
  }

  void reduce_E(int nb, int sample0, const float* partE, float* E) {
    pb();
    hipLaunchKernelGGL(k_reduce_E, dim3(blocks_for((long long)nb * c.C.K)), dim3(256), 0, st, nb, sample0,
                       c.tiles * c.waves, c.C.K, partE, E);
    pe(2);
    check("k_reduce_E");
  }

  void assemble(int seg, int nb, int sample0, const float* th, const float* xx, const float* partF, float* Gr) {
    const long long nr = (long long)(c.seg_run_begin[seg + 1] - c.seg_run_begin[seg]) * nb;
    if (nr == 0) return;
    pb();
    hipLaunchKernelGGL(k_assemble, dim3(blocks_for(nr, 128)), dim3(128), 0, st, d.tabs, seg, nb, sample0,
                       c.tiles * c.waves, c.n_angle, th, xx, c.C.F, partF, Gr);
    pe(2);
    check("k_assemble");
  }

  void reduce_grads(int nb, int sample0, const float* Gr, float* dtheta, float* dx, bool accumulate) {
    const long long total = c.C.P + (long long)nb * c.C.F;
    if (total == 0) return;
    pb();
    hipLaunchKernelGGL(k_reduce_grads, dim3(blocks_for(total)), dim3(256), 0, st, d.tabs, nb, sample0, c.n_angle,
                       c.C.P, c.C.F, Gr, dtheta, dx, accumulate ? 1 : 0);
    pe(2);
    check("k_reduce_grads");
  }

  // per-gate baseline
  void pg_init(float* psi, int nb) {
    pb();
    hipLaunchKernelGGL(k_pg_init, dim3(blocks_for(c.amps * nb)), dim3(256), 0, st, (float2*)psi, (long long)c.amps, nb);
    pe(2);
    check("k_pg_init");
  }
  void pg_copy(float* dst, const float* src, int nb) {
    if (hipMemcpyAsync(dst, src, c.state_bytes * nb, hipMemcpyDeviceToDevice, st) != hipSuccess && err == QF_OK) {
      err = QF_ERR_DEVICE;
      msg = "hipMemcpyAsync";
    }
  }
  void pg_rot(float* psi, int nb, int sample0, int r, const float* cs, const float* cp) {
    pb();
    hipLaunchKernelGGL(k_pg_rot, dim3(nb * c.pg_blocks), dim3(kPgThreads), 0, st, (float2*)psi, (long long)c.amps,
                       c.S.runs[r].q, c.S.runs[r].coef, sample0, cs, cp, c.S.n_coef_ps, c.pg_blocks);
    pe(2);
    check("k_pg_rot");
  }
  void pg_cz(float* psi, float* lam, int nb, int qa, int qb) {
    pb();
    hipLaunchKernelGGL(k_pg_cz, dim3(blocks_for((c.amps >> 2) * nb)), dim3(256), 0, st, (float2*)psi, (float2*)lam,
                       (long long)c.amps, qa, qb, nb);
    pe(2);
    check("k_pg_cz");
  }
  void pg_expect(const float* psi, int nb, float* partE) {
    pb();
    hipLaunchKernelGGL(k_pg_expect, dim3(nb * c.pg_blocks), dim3(kPgThreads), 0, st, (const float2*)psi,
                       (long long)c.amps, c.C.K, d.zmask, partE, c.pg_blocks);
    pe(2);
    check("k_pg_expect");
  }
  void pg_reduce_E(int nb, int sample0, const float* partE, float* E) {
    pb();
    hipLaunchKernelGGL(k_reduce_E, dim3(blocks_for((long long)nb * c.C.K)), dim3(256), 0, st, nb, sample0,
                       c.pg_blocks, c.C.K, partE, E);
    pe(2);
    check("k_reduce_E");
  }
  void pg_seed(const float* psi, float* lam, int nb, int sample0, const float* dE) {
    pb();
    hipLaunchKernelGGL(k_pg_seed, dim3(blocks_for(c.amps * nb)), dim3(256), 0, st, (const float2*)psi, (float2*)lam,
                       (long long)c.amps, nb, sample0, c.C.K, d.zmask, dE);
    pe(2);
    check("k_pg_seed");
  }
  void pg_rot_bwd(float* psi, float* lam, int nb, int sample0, int r, int slot, const float* cs, const float* cp,
                  float* partF) {
    pb();
    hipLaunchKernelGGL(k_pg_rot_bwd, dim3(nb * c.pg_blocks), dim3(kPgThreads), 0, st, (float2*)psi, (float2*)lam,
                       (long long)c.amps, c.S.runs[r].q, c.S.runs[r].coef, sample0, cs, cp, c.S.n_coef_ps, c.pg_blocks,
                       c.pg_chunk, slot, partF);
    pe(2);
    check("k_pg_rot_bwd");
  }
  void pg_assemble(int r0, int cnt, int nb, int sample0, const float* partF, float* Gr) {
    pb();
    hipLaunchKernelGGL(k_pg_assemble, dim3(blocks_for((long long)cnt * nb, 128)), dim3(128), 0, st, d.tabs, r0, cnt,
                       nb, c.pg_chunk, c.pg_blocks, c.n_angle, theta, x, c.C.F, sample0, partF, Gr);
    pe(2);
    check("k_pg_assemble");
  }
};

}  // namespace qf

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
using namespace qf;

struct qf_circuit {
  Circuit c;
};

struct qf_plan {
  PlanCore core;
  DevPlan dev;
  int device = 0;
  Profiler prof;
};

namespace {
thread_local std::string g_last_error;

qf_status fail(qf_status s, const std::string& m) {
  g_last_error = m;
  return s;
}
}  // namespace

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
    c->c.n = desc->n_qubits;
    c->c.P = desc->n_params;
    c->c.F = desc->n_inputs;
    c->c.K = desc->n_obs;
    c->c.gates.assign(desc->gates, desc->gates + desc->n_gates);
    c->c.obs.assign(desc->obs, desc->obs + desc->n_obs);
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
    if (T.mode != 0 && T.mode != 1) return fail(QF_ERR_INVALID_ARG, "mode must be 0 or 1");
    if (T.k < 0 || T.k > kMaxTileQubits) return fail(QF_ERR_INVALID_ARG, "tile_qubits out of range");
    if (T.R < 0 || T.R > kMaxR) return fail(QF_ERR_INVALID_ARG, "reg_qubits out of range");
    if (T.fusion < 0 || T.ckpt < 0 || T.micro < 0) return fail(QF_ERR_INVALID_ARG, "negative tuning value");
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
  info->fusion_depth = S.fusion;
  info->n_perm = S.n_perm;
  info->n_u2 = S.n_u2;
  info->n_cz = S.n_cz;
  // algorithmic bytes: every forward pass reads (except the first) and writes the
  // state once; an adjoint pass reads psi and lambda and writes lambda
  const double P = c.P;
  info->fwd_bytes_per_sample = (2 * P - 1) * SB;
  int64_t recompute = 0;
  for (int s = 0; s < c.n_seg; ++s) {
    const int a = c.seg_begin[s], b = c.seg_begin[s + 1];
    for (int q = a; q <= b - 2; ++q) recompute += (q == 0) ? 1 : 2;
  }
  const double adj = 3 * P - 2;   // the seed pass reads no lambda, pass 0 writes none
  info->bwd_pass_bytes_per_sample = adj * SB;
  info->bwd_bytes_per_sample = (recompute + adj) * SB + (c.store ? 0 : info->fwd_bytes_per_sample);
  // algorithmic flops: a 2x2 complex run on every amplitude pair is 16 real
  // multiply-adds per pair (16 flops per amplitude); the adjoint applies it to
  // psi and lambda and evaluates three functionals (6 multiply-adds per amplitude)
  const double runs = (double)S.n_u2;
  info->fwd_flops_per_sample = runs * 16 * A;
  double rec_runs = 0;
  for (int s = 0; s < c.n_seg; ++s)
    for (int q = c.seg_begin[s]; q <= c.seg_begin[s + 1] - 2; ++q) {
      const PassRec& pr = S.passes[q];
      rec_runs += pr.n_slots;
    }
  info->bwd_pass_flops_per_sample = runs * 44 * A;
  info->bwd_flops_per_sample = info->bwd_pass_flops_per_sample + rec_runs * 16 * A +
                               (c.store ? 0 : info->fwd_flops_per_sample);
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

qf_status qf_forward(qf_plan* p, const float* theta, const float* x, float* E, void* ws, size_t ws_bytes,
                     void* stream) {
  qf_status st = check_call(p, ws, ws_bytes);
  if (st != QF_OK) return st;
  const PlanCore& c = p->core;
  if (!E || (c.C.P > 0 && !theta) || (c.C.F > 0 && !x)) return fail(QF_ERR_INVALID_ARG, "NULL buffer");
  GpuExec ex(c, p->dev, (hipStream_t)stream);
  ex.prof = &p->prof;
  st = run_forward(c, ex, theta, x, E, (char*)ws);
  if (st != QF_OK) return fail(st, ex.msg);
  return QF_OK;
}

qf_status qf_backward(qf_plan* p, const float* theta, const float* x, const float* dE, float* dtheta, float* dx,
                      void* ws, size_t ws_bytes, void* stream) {
  qf_status st = check_call(p, ws, ws_bytes);
  if (st != QF_OK) return st;
  const PlanCore& c = p->core;
  if (!dE || (c.C.P > 0 && (!theta || !dtheta)) || (c.C.F > 0 && !x))
    return fail(QF_ERR_INVALID_ARG, "NULL buffer");
  GpuExec ex(c, p->dev, (hipStream_t)stream);
  ex.prof = &p->prof;
  ex.theta = theta;
  ex.x = x;
  ex.csh = (const float*)((char*)ws + c.off_coef_sh);
  ex.cps = (const float*)((char*)ws + c.off_coef_ps);
  st = run_backward(c, ex, theta, x, dE, dtheta, dx, (char*)ws);
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
