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

#include <climits>
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
  const PhaseEv* pev;
  const CzaRec* cza;
  const float* coef_sh;
  const float* coef_ps;
  const float* ev_sh;
  const float* ev_ps;
  const float2* src0;
  const float2* src1;
  float2* dst;
  float* partF;
  float* partE;
  const float* dE;
  const uint32_t* zmask;
  long long s0, s1, sd;       // per-sample strides (float2 units)
  int n_ops;
  int n_ps;                   // per-sample run coefficient rows per sample
  int n_evps;                 // per-sample phase event rows per sample
  int K;
  int sample0;
  int tiles_log2;
  int tb;                     // thread bits of the tile
  int do_expect;
  int tile_elems;             // 2^k: LDS elements of the tile; wave partial sums follow
};

// Plan tables are written before the launch and only read by it: load them
// through the constant address space so that uniform reads become scalar loads.
template <typename T>
__device__ __forceinline__ T cld(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(4))) T*)(p);
#else
  return *p;
#endif
}

// Register-bit dispatch: expands STMT with the compile-time bit J == j.
#define QF_WITH_BIT(R, j, STMT)                      \
  switch (j) {                                       \
    case 0: { constexpr int J = 0; STMT; } break;    \
    case 1: if constexpr (R > 1) { constexpr int J = 1; STMT; } break; \
    case 2: if constexpr (R > 2) { constexpr int J = 2; STMT; } break; \
    case 3: if constexpr (R > 3) { constexpr int J = 3; STMT; } break; \
    case 4: if constexpr (R > 4) { constexpr int J = 4; STMT; } break; \
    default: break;                                  \
  }

__device__ __forceinline__ uint32_t tbase(const uint32_t* tab, int t, int tb) {
  uint32_t v = 0;
#pragma unroll
  for (int i = 0; i < kMaxThreadBits; ++i)
    if (i < tb && ((t >> i) & 1)) v ^= cld(tab + i);
  return v;
}

// Per-register-bit contributions of a layout, loaded once per op (uniform).
template <int R>
struct RegBits {
  uint32_t v[R];
  __device__ __forceinline__ void load(const uint32_t* p) {
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = cld(p + j);
  }
  // XOR over the set bits of the compile-time register index jj
  __device__ __forceinline__ uint32_t operator()(int jj) const {
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < R; ++j)
      if ((jj >> j) & 1) r ^= v[j];
    return r;
  }
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// Real rotation [[c, -s], [s, c]] on the pairs along register bit J.
template <int R, int J>
__device__ __forceinline__ void apply_ry(float2 (&a)[1 << R], float c, float s) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    constexpr int m = 1 << J;
    const float2 x0 = a[i], x1 = a[i | m];
    a[i] = make_float2(fmaf(-s, x1.x, c * x0.x), fmaf(-s, x1.y, c * x0.y));
    a[i | m] = make_float2(fmaf(s, x0.x, c * x1.x), fmaf(s, x0.y, c * x1.y));
  }
}

// Diagonal phase on register bit J: w where the bit is 0, conj(w) where it is 1.
template <int R, int J>
__device__ __forceinline__ void apply_phase_reg(float2 (&a)[1 << R], float2 w) {
  const float2 wc = make_float2(w.x, -w.y);
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) a[i] = cmul(a[i], (i & (1 << J)) ? wc : w);
}

// Im<l|X_q|a>, Im<l|Y_q|a>, Im<l|Z_q|a> over the pairs along register bit J.
template <int R, int J>
__device__ __forceinline__ void func3(const float2 (&a)[1 << R], const float2 (&l)[1 << R], float& fx, float& fy,
                                      float& fz) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    constexpr int m = 1 << J;
    const float2 p0 = a[i], p1 = a[i | m], l0 = l[i], l1 = l[i | m];
    fx = fmaf(l0.x, p1.y, fx); fx = fmaf(-l0.y, p1.x, fx); fx = fmaf(l1.x, p0.y, fx); fx = fmaf(-l1.y, p0.x, fx);
    fy = fmaf(l1.x, p0.x, fy); fy = fmaf(l1.y, p0.y, fy); fy = fmaf(-l0.x, p1.x, fy); fy = fmaf(-l0.y, p1.y, fy);
    fz = fmaf(l0.x, p0.y, fz); fz = fmaf(-l0.y, p0.x, fz); fz = fmaf(-l1.x, p1.y, fz); fz = fmaf(l1.y, p1.x, fz);
  }
}

template <int NA>
__device__ __forceinline__ void scale_all(float2 (&a)[NA], float2 p) {
#pragma unroll
  for (int i = 0; i < NA; ++i) a[i] = cmul(a[i], p);
}

template <int NA>
__device__ __forceinline__ void flip_signs(float2 (&a)[NA], uint32_t sign) {
#pragma unroll
  for (int jj = 0; jj < NA; ++jj) {
    const uint32_t f = (sign << (31 - jj)) & 0x80000000u;
    a[jj].x = __uint_as_float(__float_as_uint(a[jj].x) ^ f);
    a[jj].y = __uint_as_float(__float_as_uint(a[jj].y) ^ f);
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

__device__ __forceinline__ const float* run_coef(const KArgs& A, int ref, int sample) {
  return ref >= 0 ? A.coef_sh + 8 * (size_t)ref : A.coef_ps + 8 * ((size_t)sample * A.n_ps + (-1 - ref));
}

__device__ __forceinline__ float2 event_coef(const KArgs& A, int ref, int sample) {
  const float* p = ref >= 0 ? A.ev_sh + 2 * (size_t)ref : A.ev_ps + 2 * ((size_t)sample * A.n_evps + (-1 - ref));
  return make_float2(cld(p), cld(p + 1));
}

// For register patterns jj in [0, 32): the set of jj with bit j set.
__device__ __forceinline__ uint32_t bit_pattern(int j) {
  return j == 0 ? 0xAAAAAAAAu : j == 1 ? 0xCCCCCCCCu : j == 2 ? 0xF0F0F0F0u : j == 3 ? 0xFF00FF00u : 0xFFFF0000u;
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
  const PassRec* P = A.prec;

  uint32_t tlog = 0, tin = 0, tout = 0;
  const int nnl = cld(&P->n_nonlocal);
  for (int i = 0; i < nnl; ++i)
    if ((tile >> i) & 1) {
      tlog |= 1u << cld(&P->nl_log[i]);
      tin |= 1u << cld(&P->nl_in[i]);
      tout |= 1u << cld(&P->nl_out[i]);
    }

  float2 a[NA];
  float2 l[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    a[j] = make_float2(0.f, 0.f);
    l[j] = make_float2(0.f, 0.f);
  }
  const int n_slots = cld(&P->n_slots);
  // pending per-thread phase of the diagonal gates on thread-held qubits; it
  // multiplies psi (and, in the backward, lambda as well)
  float2 ph = make_float2(1.f, 0.f);
  bool pend = false;

  // the next op record is fetched while the current one executes
  Op next = cld(A.ops);
  for (int oi = 0; oi < A.n_ops; ++oi) {
    const Op op = next;
    if (oi + 1 < A.n_ops) next = cld(A.ops + oi + 1);
    switch (op.kind) {
      case OP_INIT0: {
        const LayoutRec* L = A.layouts + op.a;
        const uint32_t base = tlog | tbase(L->log_thr, t, tb);
        RegBits<R> rb;
        rb.load(L->log_reg);
#pragma unroll
        for (int jj = 0; jj < NA; ++jj)
          a[jj] = make_float2((active && (base | rb(jj)) == 0u) ? 1.f : 0.f, 0.f);
        break;
      }
      case OP_LOAD: {
        const LayoutRec* L = A.layouts + op.a;
        const uint32_t base = (op.c ? tout : tin) | tbase(L->mem_thr, t, tb);
        RegBits<R> rb;
        rb.load(L->mem_reg);
        if (active) {
          if (op.b == 0) {
            const float2* src = A.src0 + (long long)sl * A.s0;
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) a[jj] = src[base | rb(jj)];
          } else if constexpr (BWD) {
            const float2* src = A.src1 + (long long)sl * A.s1;
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) l[jj] = src[base | rb(jj)];
          }
        }
        break;
      }
      case OP_STORE: {
        if (pend) {
          scale_all<NA>(a, ph);
          if constexpr (BWD) scale_all<NA>(l, ph);
          ph = make_float2(1.f, 0.f);
          pend = false;
        }
        const LayoutRec* L = A.layouts + op.a;
        const uint32_t base = (op.c ? tout : tin) | tbase(L->mem_thr, t, tb);
        RegBits<R> rb;
        rb.load(L->mem_reg);
        if (active && A.dst) {
          float2* dst = A.dst + (long long)sl * A.sd;
          if constexpr (BWD) {
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) dst[base | rb(jj)] = l[jj];
          } else {
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) dst[base | rb(jj)] = a[jj];
          }
        }
        break;
      }
      case OP_PERM: {
        if (pend) {
          scale_all<NA>(a, ph);
          if constexpr (BWD) scale_all<NA>(l, ph);
          ph = make_float2(1.f, 0.f);
          pend = false;
        }
        const LayoutRec* F = A.layouts + op.a;
        const LayoutRec* T = A.layouts + op.b;
        const uint32_t bf = tbase(F->lds_thr, t, tb);
        const uint32_t bt = tbase(T->lds_thr, t, tb);
        RegBits<R> rf, rt;
        rf.load(F->lds_reg);
        rt.load(T->lds_reg);
        if (active) {
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) lds[bf ^ rf(jj)] = a[jj];
        }
        __syncthreads();
        if (active) {
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) a[jj] = lds[bt ^ rt(jj)];
        }
        __syncthreads();
        if constexpr (BWD) {
          if (active) {
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) lds[bf ^ rf(jj)] = l[jj];
          }
          __syncthreads();
          if (active) {
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) l[jj] = lds[bt ^ rt(jj)];
          }
          __syncthreads();
        }
        break;
      }
      case OP_RY: {
        const float* cp = run_coef(A, op.b, sample);
        const float c = cld(cp);
        const float s = BWD ? -cld(cp + 1) : cld(cp + 1);
        if constexpr (BWD) {
          QF_WITH_BIT(R, op.a, (apply_ry<R, J>(a, c, s), apply_ry<R, J>(l, c, s)));
        } else {
          QF_WITH_BIT(R, op.a, (apply_ry<R, J>(a, c, s)));
        }
        break;
      }
      case OP_DIAGT: {
        const LayoutRec* L = A.layouts + op.a;
        const uint32_t x = tlog | tbase(L->log_thr, t, tb);
        uint32_t par = 0;
        for (int i = 0; i < op.c; ++i) {
          const CzGroup g = cld(A.czg + op.b + i);
          par ^= x & (x >> g.shift) & g.mask;
        }
        const uint32_t f = (uint32_t)(__popc(par) & 1) << 31;
        ph.x = __uint_as_float(__float_as_uint(ph.x) ^ f);
        ph.y = __uint_as_float(__float_as_uint(ph.y) ^ f);
        for (int i = 0; i < op.e; ++i) {
          const PhaseEv e = cld(A.pev + op.d + i);
          float2 w = event_coef(A, e.ref, sample);
          const bool conj = (((x >> e.q) & 1u) != 0u) != BWD;
          if (conj) w.y = -w.y;
          ph = cmul(ph, w);
        }
        pend = true;
        break;
      }
      case OP_CZA: {
        const CzaRec* C = A.cza + op.a;
        const LayoutRec* L = A.layouts + op.b;
        const uint32_t x = tlog | tbase(L->log_thr, t, tb);
        uint32_t sign = cld(&C->sr);
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (__popc(x & cld(&C->cmask[j])) & 1) sign ^= bit_pattern(j);
        flip_signs<NA>(a, sign);
        if constexpr (BWD) flip_signs<NA>(l, sign);
        break;
      }
      case OP_PHASEA: {
        const PhaseEv e = cld(A.pev + op.b);
        float2 w = event_coef(A, e.ref, sample);
        if (BWD) w.y = -w.y;
        if constexpr (BWD) {
          QF_WITH_BIT(R, op.a, (apply_phase_reg<R, J>(a, w), apply_phase_reg<R, J>(l, w)));
        } else {
          QF_WITH_BIT(R, op.a, (apply_phase_reg<R, J>(a, w)));
        }
        break;
      }
      case OP_EXPECT: {
        if constexpr (!BWD) {
          if (!A.do_expect) break;
          const LayoutRec* L = A.layouts + op.a;
          const uint32_t base = tlog | tbase(L->log_thr, t, tb);
          RegBits<R> rb;
          rb.load(L->log_reg);
          for (int k0 = 0; k0 < A.K; k0 += 16) {
            float v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = 0.f;
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) {
              const uint32_t x = base | rb(jj);
              const float p = fmaf(a[jj].x, a[jj].x, a[jj].y * a[jj].y);
#pragma unroll
              for (int k = 0; k < 16; ++k)
                if (k0 + k < A.K) v[k] += (__popc(x & cld(A.zmask + k0 + k)) & 1) ? -p : p;
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
          const LayoutRec* L = A.layouts + op.a;
          const uint32_t base = tlog | tbase(L->log_thr, t, tb);
          RegBits<R> rb;
          rb.load(L->log_reg);
          const float* g = A.dE + (size_t)sample * A.K;
          // lambda = 2 c(x) psi, c(x) = sum_k g_k (-1)^{|x & z_k|}
          float c[NA];
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) c[jj] = 0.f;
#pragma unroll 1
          for (int k = 0; k < A.K; ++k) {
            const float gk = cld(g + k);
            const uint32_t zk = cld(A.zmask + k);
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) c[jj] += (__popc((base | rb(jj)) & zk) & 1) ? -gk : gk;
          }
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) l[jj] = make_float2(2.f * c[jj] * a[jj].x, 2.f * c[jj] * a[jj].y);
        }
        break;
      }
      case OP_FUNC: {
        if constexpr (BWD) {
          const FuncEntry* fe = A.funcs + op.b;
          const int m = op.a;
          float v[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) v[i] = 0.f;
#pragma unroll 1
          for (int e = 0; e < m; ++e) {
            float fx = 0.f, fy = 0.f, fz = 0.f;
            const int rb = cld(&fe[e].regbit);
            QF_WITH_BIT(R, rb, (func3<R, J>(a, l, fx, fy, fz)));
            // place the three sums of entry e (static register indices)
#pragma unroll
            for (int q = 0; q < R; ++q)
              if (q == e) {
                v[3 * q] = fx;
                v[3 * q + 1] = fy;
                v[3 * q + 2] = fz;
              }
          }
          const float s = wave_reduce16(v, lane);
          const int idx = (lane >> 2) & 15;
          if ((lane & 3) == 0 && idx < 3 * m) {
            const int e = idx / 3, pq = idx - 3 * e;
            float* part = reinterpret_cast<float*>(lds + A.tile_elems);
            part[wave * 3 * n_slots + 3 * fe[e].slot + pq] = s;
          }
        }
        break;
      }
      default:
        break;
    }
  }
  if constexpr (BWD) {
    // one partial sum per tile and functional: add the waves' sums
    if (n_slots > 0) {
      __syncthreads();
      const float* part = reinterpret_cast<const float*>(lds + A.tile_elems);
      for (int i = t; i < 3 * n_slots; i += NT) {
        float acc = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) acc += part[w * 3 * n_slots + i];
        A.partF[(size_t)item * 3 * n_slots + i] = acc;
      }
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
  const EventRec* events;
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
  const int32_t* pass_run_begin;
  const int32_t* pass_runs;
};

__device__ inline double gate_angle(const GateRec& g, const float* theta, const float* x, int F, int sample) {
  return g.theta_idx >= 0 ? (double)theta[g.theta_idx] : (double)x[(size_t)sample * F + g.input_idx];
}

// RZ(a) RY(b) RZ(c) split of an SU(2) matrix V (V00 = e^{-i(a+c)/2} cos(b/2),
// V10 = e^{i(a-c)/2} sin(b/2)).  Returns cos(b/2), sin(b/2), u = e^{-ia/2},
// v = e^{-ic/2} and z = u^2 = e^{-ia}.
struct ZYZ {
  double cb, sb, ur, ui, vr, vi, zr, zi;
};

__device__ inline ZYZ zyz_split(const D2& V) {
  ZYZ o;
  const double a0 = sqrt(V.r[0] * V.r[0] + V.i[0] * V.i[0]);
  const double b0 = sqrt(V.r[2] * V.r[2] + V.i[2] * V.i[2]);
  const double nrm = sqrt(a0 * a0 + b0 * b0);
  o.cb = a0 / nrm;
  o.sb = b0 / nrm;
  double Ar = 1, Ai = 0, Br = 1, Bi = 0;
  if (a0 > 1e-300) { Ar = V.r[0] / a0; Ai = V.i[0] / a0; }
  if (b0 > 1e-300) { Br = V.r[2] / b0; Bi = V.i[2] / b0; }
  o.zr = Ar * Br + Ai * Bi;        // A conj(B)
  o.zi = Ai * Br - Ar * Bi;
  const double th = atan2(o.zi, o.zr);
  double s, c;
  sincos(0.5 * th, &s, &c);
  o.ur = c;
  o.ui = s;
  o.vr = Ar * c + Ai * s;          // A conj(u)
  o.vi = Ai * c - Ar * s;
  return o;
}

__device__ inline D2 run_matrix(const Tabs& T, const RunRec& rr, const float* theta, const float* x, int F,
                                int sample) {
  D2 U = d2_eye();
  for (int i = 0; i < rr.gate_count; ++i) {
    const GateRec g = T.gates[T.run_gates[rr.gate_begin + i]];
    U = d2_mul(d2_rot(g.kind, gate_angle(g, theta, x, F, sample)), U);
  }
  return U;
}

// Run coefficients.  zyz = 1: [cos(b/2), sin(b/2), u, v] of the RZ RY RZ split;
// zyz = 0: the 2x2 matrix row-major (one-gate runs of the per-gate baseline).
__global__ void k_coef(Tabs T, const float* theta, const float* x, int F, int n_sh, int n_ps, int B, float* csh,
                       float* cps, int zyz) {
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
  const D2 U = run_matrix(T, T.runs[r], theta, x, F, sample);
  if (zyz) {
    const ZYZ z = zyz_split(U);
    out[0] = (float)z.cb; out[1] = (float)z.sb;
    out[2] = (float)z.ur; out[3] = (float)z.ui;
    out[4] = (float)z.vr; out[5] = (float)z.vi;
    out[6] = 0.f; out[7] = 0.f;
  } else {
    for (int i = 0; i < 4; ++i) {
      out[2 * i] = (float)U.r[i];
      out[2 * i + 1] = (float)U.i[i];
    }
  }
}

// Phase event coefficients w = u(prev run) * v(next run).
__global__ void k_event_coef(Tabs T, int n_ev_sh, int n_ev_ps, int B, int n_ps, const float* csh, const float* cps,
                             float* esh, float* eps) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = n_ev_sh + (long long)n_ev_ps * B;
  if (idx >= total) return;
  int sample = 0;
  EventRec e;
  float* out;
  if (idx < n_ev_sh) {
    e = T.events[idx];
    out = esh + 2 * idx;
  } else {
    const long long j = idx - n_ev_sh;
    sample = (int)(j / n_ev_ps);
    const int i = (int)(j - (long long)sample * n_ev_ps);
    e = T.events[n_ev_sh + i];
    out = eps + 2 * j;
  }
  auto row = [&](int ref) {
    return ref >= 0 ? csh + 8 * (long long)ref : cps + 8 * ((long long)sample * n_ps + (-1 - ref));
  };
  float wr = 1.f, wi = 0.f;
  if (e.prev_ref != INT32_MIN) {
    const float* p = row(e.prev_ref);
    const float ur = p[2], ui = p[3];
    const float tr = wr * ur - wi * ui, ti = wr * ui + wi * ur;
    wr = tr; wi = ti;
  }
  if (e.next_ref != INT32_MIN) {
    const float* p = row(e.next_ref);
    const float vr = p[4], vi = p[5];
    const float tr = wr * vr - wi * vi, ti = wr * vi + wi * vr;
    wr = tr; wi = ti;
  }
  out[0] = wr;
  out[1] = wi;
}

// Gradients of the gates of run r from the functionals F = Im<lambda|P_q|psi>
// (P = X, Y, Z) taken at the cut right after the run's RY (zyz = 1) or right
// after the whole run (zyz = 0).  dL/dtheta_g = 1/2 Im<lambda|G|psi>, with G the
// generator of gate g carried to the cut: G = K P_g K^dagger (K = gates of the
// run after g), conjugated by RZ(a)^dagger for the zyz cut.  Writing
// G = n_x X + n_y Y + n_z Z gives dL/dtheta_g = 1/2 (n . F).
__device__ inline void run_grads(const Tabs& T, int r, const float* theta, const float* x, int F, int sample,
                                 double fx, double fy, double fz, float* Grow, int zyz) {
  const RunRec rr = T.runs[r];
  double zr = 1, zi = 0;
  if (zyz) {
    const ZYZ z = zyz_split(run_matrix(T, rr, theta, x, F, sample));
    zr = z.zr;
    zi = z.zi;
  }
  D2 K = d2_eye();
  for (int i = rr.gate_count - 1; i >= 0; --i) {
    const GateRec g = T.gates[T.run_gates[rr.gate_begin + i]];
    const D2 G = d2_mul(d2_mul(K, d2_pauli(g.kind)), d2_dag(K));
    const double gr = zr * G.r[2] - zi * G.i[2], gi = zr * G.i[2] + zi * G.r[2];
    Grow[g.out_idx] = (float)(0.5 * (gr * fx + gi * fy + G.r[0] * fz));
    K = d2_mul(K, d2_rot(g.kind, gate_angle(g, theta, x, F, sample)));
  }
}

// One block per (sample, pass of the segment): sum the pass's per-tile
// functional partials (coalesced over the slots), then one thread per run turns
// the three sums into the run's per-gate gradients.
__global__ __launch_bounds__(256) void k_assemble(Tabs T, int p0, int np, int nb, int sample0, int tiles,
                                                  int n_angle, const float* theta, const float* x, int F,
                                                  const float* partF, float* Gr) {
  extern __shared__ double fsum[];
  const int s = blockIdx.x / np, p = p0 + (int)(blockIdx.x - s * np);
  const int ns = T.passes[p].n_slots;
  if (ns == 0) return;
  const float* base = partF + (long long)nb * T.partF_off[p] + (long long)s * tiles * 3 * ns;
  for (int v = threadIdx.x; v < 3 * ns; v += blockDim.x) {
    double acc = 0;
    for (int tile = 0; tile < tiles; ++tile) acc += base[(long long)tile * 3 * ns + v];
    fsum[v] = acc;
  }
  __syncthreads();
  const int rb = T.pass_run_begin[p];
  for (int i = threadIdx.x; i < ns; i += blockDim.x)
    run_grads(T, T.pass_runs[rb + i], theta, x, F, sample0 + s, fsum[3 * i], fsum[3 * i + 1], fsum[3 * i + 2],
              Gr + (long long)s * n_angle, 1);
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
  run_grads(T, r, theta, x, F, sample0 + s, f[0], f[1], f[2], Gr + (long long)s * n_angle, 0);
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
  const PhaseEv* pev = nullptr;
  const CzaRec* cza = nullptr;
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
  push_table(blob, o, c.S.pev);          // 18
  push_table(blob, o, c.S.cza);          // 19
  push_table(blob, o, c.S.events);       // 20
  push_table(blob, o, c.S.pass_run_begin);  // 21
  push_table(blob, o, c.S.pass_runs);    // 22
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
  d->pev = (const PhaseEv*)(b + o[18]);
  d->cza = (const CzaRec*)(b + o[19]);
  t.events = (const EventRec*)(b + o[20]);
  t.pass_run_begin = (const int32_t*)(b + o[21]);
  t.pass_runs = (const int32_t*)(b + o[22]);
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

  const float* esh = nullptr;
  const float* eps = nullptr;
  void coef(const float* th, const float* xx, char* ws) {
    theta = th; x = xx;
    float* cs = at<float>(ws, c.off_coef_sh);
    float* cp = at<float>(ws, c.off_coef_ps);
    float* es = at<float>(ws, c.off_ev_sh);
    float* ep = at<float>(ws, c.off_ev_ps);
    csh = cs; cps = cp; esh = es; eps = ep;
    const long long total = c.S.n_coef_shared + (long long)c.S.n_coef_ps * c.B;
    if (total > 0) {
      pb();
      hipLaunchKernelGGL(k_coef, dim3(blocks_for(total)), dim3(256), 0, st, d.tabs, th, xx, c.C.F, c.S.n_coef_shared,
                         c.S.n_coef_ps, c.B, cs, cp, c.per_gate ? 0 : 1);
      pe(2);
      check("k_coef");
    }
    const long long ne = c.S.n_ev_shared + (long long)c.S.n_ev_ps * c.B;
    if (ne > 0) {
      pb();
      hipLaunchKernelGGL(k_event_coef, dim3(blocks_for(ne)), dim3(256), 0, st, d.tabs, c.S.n_ev_shared,
                         c.S.n_ev_ps, c.B, c.S.n_coef_ps, cs, cp, es, ep);
      pe(2);
      check("k_event_coef");
    }
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
    A.pev = d.pev;
    A.cza = d.cza;
    A.coef_sh = csh;
    A.coef_ps = cps;
    A.ev_sh = esh;
    A.ev_ps = eps;
    A.n_ps = S.n_coef_ps;
    A.n_evps = S.n_ev_ps;
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
    A.tile_elems = 1 << S.k;
    const size_t shmem = (sizeof(float2) << S.k) + (L.bwd ? sizeof(float) * 3 * S.max_slots * S.NT / 64 : 0);
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
    const int p0 = c.seg_begin[seg], np = c.seg_begin[seg + 1] - p0;
    if (np == 0 || nb == 0) return;
    pb();
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)(nb * np)), dim3(256), sizeof(double) * 3 * std::max(1, c.S.max_slots),
                       st, d.tabs, p0, np, nb, sample0, c.tiles, c.n_angle, th, xx, c.C.F, partF, Gr);
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
  // algorithmic flops of a run: its real RY on every complex amplitude pair is 8
  // multiply-adds per pair (8 flops per amplitude); the adjoint applies RY^dagger
  // to psi and lambda (16 flops per amplitude) and evaluates the three
  // functionals (6 multiply-adds, 12 flops per amplitude)
  const double runs = (double)S.n_u2;
  info->fwd_flops_per_sample = runs * 8 * A;
  double rec_runs = 0;
  for (int s = 0; s < c.n_seg; ++s)
    for (int q = c.seg_begin[s]; q <= c.seg_begin[s + 1] - 2; ++q) {
      const PassRec& pr = S.passes[q];
      rec_runs += pr.n_slots;
    }
  info->bwd_pass_flops_per_sample = runs * 28 * A;
  info->bwd_flops_per_sample = info->bwd_pass_flops_per_sample + rec_runs * 8 * A +
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
  ex.esh = (const float*)((char*)ws + c.off_ev_sh);
  ex.eps = (const float*)((char*)ws + c.off_ev_ps);
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
