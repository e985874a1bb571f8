// device.hpp -- device code of the fused pass kernels, shared by the
// single-plan kernels and the merged mixed-batch kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

#include "kargs.hpp"

namespace qf {

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

// Plan records, read field by field so that every field is a scalar load
// (whole-struct reads through the constant address space can turn into vector
// loads followed by a wait on the vector memory counter).
__device__ __forceinline__ Op ld_op(const Op* p) {
  Op o;
  o.kind = cld(&p->kind);
  o.a = cld(&p->a);
  o.b = cld(&p->b);
  o.c = cld(&p->c);
  o.d = cld(&p->d);
  o.e = cld(&p->e);
  o.f = 0;
  o.g = 0;
  return o;
}

__device__ __forceinline__ PhaseEv ld_pev(const PhaseEv* p) {
  PhaseEv e;
  e.q = cld(&p->q);
  e.ref = cld(&p->ref);
  return e;
}

__device__ __forceinline__ CzGroup ld_czg(const CzGroup* p) {
  CzGroup g;
  g.shift = cld(&p->shift);
  g.mask = cld(&p->mask);
  return g;
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

// log2 of the threads of a workgroup (a tile with fewer thread bits leaves lanes idle)
template <int NT>
struct ThreadBitsOf {
  static constexpr int value = NT <= 64 ? 6 : NT <= 128 ? 7 : 8;
};

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

// a *= b, ordered so that each new component is produced by the last use of
// the old one (both can then share a register: loop-carried register arrays
// stay in place instead of being copied every iteration).
__device__ __forceinline__ void cmul_in(float2& a, float2 b) {
  const float t1 = a.y * b.y;
  const float t2 = a.y * b.x;
  a.y = fmaf(a.x, b.y, t2);
  a.x = fmaf(a.x, b.x, -t1);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// Real rotation [[cos f, -sin f], [sin f, cos f]] on the pairs along register
// bit J, as three shears (x0 -= t x1; x1 += s x0; x0 -= t x1 with t = tan(f/2),
// s = sin f): three fused multiply-adds per real pair, computed in place.  The
// run coefficients keep f in [0, pi/2], so |t|, |s| <= 1.
template <int R, int J>
__device__ __forceinline__ void apply_ry(float2 (&a)[1 << R], float t, float s) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    constexpr int m = 1 << J;
    a[i].x = fmaf(-t, a[i | m].x, a[i].x);
    a[i].y = fmaf(-t, a[i | m].y, a[i].y);
    a[i | m].x = fmaf(s, a[i].x, a[i | m].x);
    a[i | m].y = fmaf(s, a[i].y, a[i | m].y);
    a[i].x = fmaf(-t, a[i | m].x, a[i].x);
    a[i].y = fmaf(-t, a[i | m].y, a[i].y);
  }
}

// RY on every register bit, bits 0..R-1 in order, straight-line code.
template <int R, int J = 0>
__device__ __forceinline__ void apply_ry_all(float2 (&a)[1 << R], const float (&t)[R], const float (&s)[R]) {
  if constexpr (J < R) {
    apply_ry<R, J>(a, t[J], s[J]);
    apply_ry_all<R, J + 1>(a, t, s);
  }
}

// Diagonal phase on register bit J: w where the bit is 0, conj(w) where it is 1.
template <int R, int J>
__device__ __forceinline__ void apply_phase_reg(float2 (&a)[1 << R], float2 w) {
  const float2 wc = make_float2(w.x, -w.y);
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) cmul_in(a[i], (i & (1 << J)) ? wc : w);
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

// Functionals of every register bit, bits 0..R-1 in order, into v[3J..3J+2].
template <int R, int J = 0>
__device__ __forceinline__ void func3_all(const float2 (&a)[1 << R], const float2 (&l)[1 << R], float (&v)[16]) {
  if constexpr (J < R) {
    func3<R, J>(a, l, v[3 * J], v[3 * J + 1], v[3 * J + 2]);
    func3_all<R, J + 1>(a, l, v);
  }
}

// Im<l|X_q|a> and Im<l|Y_q|a> over the pairs along register bit J (the terms
// couple the two amplitudes of a pair: eight fused multiply-adds per pair).
template <int R, int J>
__device__ __forceinline__ void func_xy(const float2 (&a)[1 << R], const float2 (&l)[1 << R], float& fx, float& fy) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    constexpr int m = 1 << J;
    const float2 p0 = a[i], p1 = a[i | m], l0 = l[i], l1 = l[i | m];
    fx = fmaf(l0.x, p1.y, fx); fx = fmaf(-l0.y, p1.x, fx); fx = fmaf(l1.x, p0.y, fx); fx = fmaf(-l1.y, p0.x, fx);
    fy = fmaf(l1.x, p0.x, fy); fy = fmaf(l1.y, p0.y, fy); fy = fmaf(-l0.x, p1.x, fy); fy = fmaf(-l0.y, p1.y, fy);
  }
}

// Im<l|Z_q|a> of every register bit q.  Z is diagonal, so with u_i = Im(conj(l_i) a_i)
// per slot the functional of bit J is sum_i (-1)^(bit J of i) u_i, i.e. twice the sum
// over the slots with bit J clear minus the sum over all slots.  The slots are added
// pairwise along bit 0, then along bit 1, and so on; before the additions along bit J
// the entries with bit J clear are the even ones.  62 instructions for R = 4, against
// 128 fused multiply-adds when each bit sums its pairs on its own.
template <int R>
__device__ __forceinline__ void func_z_all(const float2 (&a)[1 << R], const float2 (&l)[1 << R], float (&z)[R]) {
  // level 0 streamed from the slots: u of each pair, the even-slot sum and the pair sums
  float w[(1 << R) / 2];
  float ev[R];
#pragma unroll
  for (int k = 0; k < (1 << R) / 2; ++k) {
    const float u0 = fmaf(l[2 * k].x, a[2 * k].y, -(l[2 * k].y * a[2 * k].x));
    const float u1 = fmaf(l[2 * k + 1].x, a[2 * k + 1].y, -(l[2 * k + 1].y * a[2 * k + 1].x));
    ev[0] = k == 0 ? u0 : ev[0] + u0;
    w[k] = u0 + u1;
  }
#pragma unroll
  for (int j = 1; j < R; ++j) {
    const int n = (1 << R) >> j;
    float e = w[0];
#pragma unroll
    for (int m = 2; m < n; m += 2) e += w[m];
    ev[j] = e;
#pragma unroll
    for (int m = 0; m < n / 2; ++m) w[m] = w[2 * m] + w[2 * m + 1];
  }
  // w[0]: the sum over all slots
#pragma unroll
  for (int j = 0; j < R; ++j) z[j] = fmaf(2.f, ev[j], -w[0]);
}

template <int R, int J = 0>
__device__ __forceinline__ void func_xy_all(const float2 (&a)[1 << R], const float2 (&l)[1 << R], float (&v)[3 * R]) {
  if constexpr (J < R) {
    func_xy<R, J>(a, l, v[3 * J], v[3 * J + 1]);
    func_xy_all<R, J + 1>(a, l, v);
  }
}

template <int NA>
__device__ __forceinline__ void scale_all(float2 (&a)[NA], float2 p) {
#pragma unroll
  for (int i = 0; i < NA; ++i) cmul_in(a[i], p);
}

template <int NA>
__device__ __forceinline__ void flip_signs(float2 (&a)[NA], uint32_t sign) {
  // negation of slot jj where bit jj of sign is set, as an XOR of the float
  // sign bits (exact; no compare or select)
#pragma unroll
  for (int jj = 0; jj < NA; ++jj) {
    const uint32_t m = (sign << (31 - jj)) & 0x80000000u;
    a[jj].x = __uint_as_float(__float_as_uint(a[jj].x) ^ m);
    a[jj].y = __uint_as_float(__float_as_uint(a[jj].y) ^ m);
  }
}

// Cross-lane moves of one float (DPP, no LDS traffic).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]: lane ^ 1
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]: lane ^ 2
constexpr int kDppRowRor4 = 0x124;   // row_ror:4 (rows of 16 lanes)
constexpr int kDppRowRor8 = 0x128;   // row_ror:8: lane ^ 8 inside a row

// x (lanes whose bit is clear) or y (lanes whose bit is set), each summed with
// the same value of the partner lane across that bit
__device__ __forceinline__ float sum_split(float x, float y, float xp, float yp, bool hi) {
  return hi ? y + yp : x + xp;
}

// Reduce-scatter of 16 per-lane values over a wave of 64 lanes.  Afterwards
// every lane holds the wave sum of value wave_sum_index(lane).  Lane bits 5 and
// 4 are folded with v_permlane32_swap / v_permlane16_swap (one swap and one add
// per pair of values), bits 0 and 1 with quad DPP moves, and the last value is
// summed over bits 3 and 2 with row rotations; no LDS instruction is issued.
__device__ __forceinline__ float wave_reduce16(float (&v)[16], int lane) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    // the upper half of v[i] and the lower half of v[i + 8] change places: the
    // lower lanes then hold both halves of v[i], the upper lanes both of v[i + 8]
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 8]), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    // odd rows of v[i] with even rows of v[i + 4]
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 4]), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  {
    const bool hi = (lane & 1) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
      v[i] = sum_split(v[i], v[i + 2], dpp_mov<kDppQuadXor1>(v[i]), dpp_mov<kDppQuadXor1>(v[i + 2]), hi);
  }
  {
    const bool hi = (lane & 2) != 0;
    v[0] = sum_split(v[0], v[1], dpp_mov<kDppQuadXor2>(v[0]), dpp_mov<kDppQuadXor2>(v[1]), hi);
  }
  // full sums over lane bits 3 and 2: lane ^ 8 inside a row; then a rotation by 4,
  // which reaches lane ^ 4 once the values no longer depend on bit 3
  v[0] += dpp_mov<kDppRowRor8>(v[0]);
  v[0] += dpp_mov<kDppRowRor4>(v[0]);
  return v[0];
}

// Index of the value whose wave sum lane `lane` holds after wave_reduce16; the
// lanes with bits 2 and 3 clear hold each index once.
__device__ __forceinline__ int wave_sum_index(int lane) {
  return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + (lane & 1) * 2 + ((lane >> 1) & 1);
}
__device__ __forceinline__ bool wave_sum_writer(int lane) { return (lane & 12) == 0; }

// Reduce-scatter of 12 per-lane values (the three functionals of four register
// bits) over a wave of 64 lanes.  Lane bit 5 pairs v[i] with v[i + 6] and lane bit
// 4 pairs v[i] with v[i + 3] (one permlane swap and one add per pair); lane bit 0
// splits v[0] from v[1] and sums v[2] whole, lane bit 1 splits those two results,
// and lane bits 3 and 2 are summed whole.  Afterwards every lane holds the wave sum
// of value wave_sum_index12(lane); 27 instructions, against 43 for the 16-value
// reduction padded with zeros.
__device__ __forceinline__ float wave_reduce12(float (&v)[12], int lane) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 6]), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 3]), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  {
    const bool hi = (lane & 1) != 0;
    v[0] = sum_split(v[0], v[1], dpp_mov<kDppQuadXor1>(v[0]), dpp_mov<kDppQuadXor1>(v[1]), hi);
    v[1] = v[2] + dpp_mov<kDppQuadXor1>(v[2]);
  }
  {
    const bool hi = (lane & 2) != 0;
    v[0] = sum_split(v[0], v[1], dpp_mov<kDppQuadXor2>(v[0]), dpp_mov<kDppQuadXor2>(v[1]), hi);
  }
  v[0] += dpp_mov<kDppRowRor8>(v[0]);
  v[0] += dpp_mov<kDppRowRor4>(v[0]);
  return v[0];
}

// Value whose wave sum lane `lane` holds after wave_reduce12: 3 * e + p with e =
// lane bits 5,4 (the register bit) and p = 2 where lane bit 1 is set, else lane
// bit 0 (the Pauli); the writer lanes (bits 2 and 3 clear, not both of bits 0 and
// 1 set) hold each value once.
__device__ __forceinline__ int wave_sum_pauli12(int lane) { return (lane & 2) ? 2 : (lane & 1); }
__device__ __forceinline__ bool wave_sum_writer12(int lane) { return (lane & 12) == 0 && (lane & 3) != 3; }

__device__ __forceinline__ const float* run_coef(const KArgs& A, int ref, int sample) {
  return ref >= 0 ? A.coef_sh + 8 * (size_t)ref : A.coef_ps + 8 * ((size_t)sample * A.n_ps + (-1 - ref));
}

__device__ __forceinline__ float2 event_coef(const KArgs& A, int ref, int sample) {
  // shared row ref >= 0, or per-sample row -1 - ref: selected without a branch
  const bool sh = ref >= 0;
  const float* base = sh ? A.ev_sh : A.ev_ps + 2 * (size_t)sample * A.n_evps;
  const float* p = base + 2 * (size_t)(sh ? ref : -1 - ref);
  return make_float2(cld(p), cld(p + 1));
}

// Memory-saving storage of an amplitude: real and imaginary parts as two
// bfloat16 in one word (round to nearest even, real part in the low half), and
// the exact widening back to float.
typedef __bf16 qf_bf16x2 __attribute__((ext_vector_type(2)));
typedef float qf_f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float2 v) {
  const qf_f32x2 f = {v.x, v.y};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, qf_bf16x2));
}
__device__ __forceinline__ float2 widen_bf16x2(uint32_t u) {
  return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
}

// LDS amplitude at a byte offset (layouts hold LDS positions in bytes).
__device__ __forceinline__ float2& lds_at(float2* lds, uint32_t byte_off) {
  return *reinterpret_cast<float2*>(reinterpret_cast<char*>(lds) + byte_off);
}

// For register patterns jj in [0, 32): the set of jj with bit j set.
__device__ __forceinline__ uint32_t bit_pattern(int j) {
  return j == 0 ? 0xAAAAAAAAu : j == 1 ? 0xCCCCCCCCu : j == 2 ? 0xF0F0F0F0u : j == 3 ? 0xFF00FF00u : 0xFFFF0000u;
}

// Minimum waves per SIMD the pass kernels are compiled for (bounds registers).
template <int R, bool BWD>
constexpr int pass_min_waves() {
  return R <= 4 ? 3 : 1;
}

// Backward pass workgroups: one functional partial sum per wave, slot and Pauli
// (dynamic LDS after the static tile).
extern __shared__ float qf_pass_part[];

// Per-workgroup context of a fused pass: the uniform launch arguments, the
// thread's coordinates and the bodies of the ops.  The register arrays and the
// pending phase are passed by reference, so that they stay in registers.
template <int R, int NT, bool BWD>
struct PassCtx {
  static constexpr int NA = 1 << R;
  static constexpr int WAVES = NT / 64;
  KArgs A;
  float2* lds;
  int t;
  uint32_t tlog;
  bool active;
  int sample, lane, wave, n_slots;

  // The thread's {LDS offset, logical index} bases of a layout, read from the
  // plan's per-thread table (a vector load through the caches).
  __device__ __forceinline__ uint2 base2(int layout) const {
    return *reinterpret_cast<const uint2*>(A.tbases + ((size_t)layout * NT + t));
  }
  __device__ __forceinline__ uint32_t mem_base(int layout) const {
    return A.tbases[(size_t)layout * NT + t].mem;
  }
  // logical base of `layout`, reusing the bases `cur` of layout `cur_idx` when they match
  __device__ __forceinline__ uint32_t log_base(int layout, int cur_idx, uint2 cur) const {
    return tlog | (layout == cur_idx ? cur.y : base2(layout).y);
  }

  // op bodies, shared by the single ops and the fused epoch op.  bf, bt: the
  // thread's LDS bases of the layouts before and after the exchange.
  __device__ __forceinline__ void perm(float2 (&a)[NA], float2 (&l)[NA], float2& ph, int from, int to,
                                       uint32_t bf, uint32_t bt) const {
  // flush the pending phase (an exact identity when none is pending)
  scale_all<NA>(a, ph);
  if constexpr (BWD) scale_all<NA>(l, ph);
  ph = make_float2(1.f, 0.f);
  const LayoutRec* F = A.layouts + from;
  const LayoutRec* T = A.layouts + to;
  RegBits<R> rf, rt;
  rf.load(F->lds_reg);
  rt.load(T->lds_reg);
  if (active) {
#pragma unroll
    for (int jj = 0; jj < NA; ++jj) lds_at(lds, bf ^ rf(jj)) = a[jj];
  }
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < NA; ++jj) a[jj] = lds_at(lds, bt ^ rt(jj));
  __syncthreads();
  if constexpr (BWD) {
    if (active) {
#pragma unroll
      for (int jj = 0; jj < NA; ++jj) lds_at(lds, bf ^ rf(jj)) = l[jj];
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < NA; ++jj) l[jj] = lds_at(lds, bt ^ rt(jj));
    __syncthreads();
  }
  }

  // RY(b) as a rotation by f = b/2: shear coefficients tan(f/2), sin f; the
  // backward un-applies it (f -> -f)
  __device__ __forceinline__ void ry(float2 (&a)[NA], float2 (&l)[NA], float2& ph, int bit, int ref) const {
    // one run: the group code with identity coefficients on the other bits
    const float* cp = run_coef(A, ref, sample);
    const float t0 = BWD ? -cld(cp + 6) : cld(cp + 6);
    const float s0 = BWD ? -cld(cp + 1) : cld(cp + 1);
    float tt[R], sn[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      tt[j] = (j == bit) ? t0 : 0.f;
      sn[j] = (j == bit) ? s0 : 0.f;
    }
    apply_ry_all<R>(a, tt, sn);
    if constexpr (BWD) apply_ry_all<R>(l, tt, sn);
  }
  __device__ __forceinline__ void ryg(float2 (&a)[NA], float2 (&l)[NA], float2& ph, int first, int mask) const {
  const RygEntry* ge = A.rygs + first;
  float tt[R], sn[R];
  int e = 0;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    tt[j] = 0.f;
    sn[j] = 0.f;
    if ((mask >> j) & 1) {
      const float* cp = run_coef(A, cld(&ge[e].ref), sample);
      tt[j] = BWD ? -cld(cp + 6) : cld(cp + 6);
      sn[j] = BWD ? -cld(cp + 1) : cld(cp + 1);
      ++e;
    }
  }
  apply_ry_all<R>(a, tt, sn);
  if constexpr (BWD) apply_ry_all<R>(l, tt, sn);
  }

  // x: the thread's logical base index in the current layout
  __device__ __forceinline__ void diagt(float2 (&a)[NA], float2 (&l)[NA], float2& ph, uint32_t x, int czg0, int nczg, int pev0, int npev) const {
  uint32_t par = 0;
  for (int i = 0; i < nczg; ++i) {
    const CzGroup g = ld_czg(A.czg + czg0 + i);
    par ^= x & (x >> g.shift) & g.mask;
  }
  const uint32_t f = (uint32_t)(__popc(par) & 1) << 31;
  const float g = f ? -1.f : 1.f;
  ph.x *= g;
  ph.y *= g;
  // phase events in groups of four: the records, then the coefficients, are
  // loaded together, so that each group waits on scalar memory twice
  int i = 0;
  for (; i + 4 <= npev; i += 4) {
    PhaseEv e[4];
    float2 w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = ld_pev(A.pev + pev0 + i + k);
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = event_coef(A, e[k].ref, sample);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // conjugate where the event's qubit is 1 (0 in the backward): sign-bit XOR
      w[k].y = __uint_as_float(__float_as_uint(w[k].y) ^ (((x >> e[k].q) << 31) ^ (BWD ? 0x80000000u : 0u)));
      cmul_in(ph, w[k]);
    }
  }
  for (; i < npev; ++i) {
    const PhaseEv e = ld_pev(A.pev + pev0 + i);
    float2 w = event_coef(A, e.ref, sample);
    w.y = __uint_as_float(__float_as_uint(w.y) ^ (((x >> e.q) << 31) ^ (BWD ? 0x80000000u : 0u)));
    cmul_in(ph, w);
  }
  }

  __device__ __forceinline__ void cza(float2 (&a)[NA], float2 (&l)[NA], float2& ph, int cza, uint32_t x) const {
  const CzaRec* C = A.cza + cza;
  uint32_t sign = cld(&C->sr);
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (__popc(x & cld(&C->cmask[j])) & 1) sign ^= bit_pattern(j);
  flip_signs<NA>(a, sign);
  if constexpr (BWD) flip_signs<NA>(l, sign);
  }

  __device__ __forceinline__ void phasea(float2 (&a)[NA], float2 (&l)[NA], float2& ph, int bit, int pev) const {
    // diag(w, conj w) on register bit `bit`: the factor of slot jj is chosen
    // with a uniform select, so no code depends on the bit at compile time
    const PhaseEv e = ld_pev(A.pev + pev);
    float2 w = event_coef(A, e.ref, sample);
    if (BWD) w.y = -w.y;
    const float2 wc = make_float2(w.x, -w.y);
#pragma unroll
    for (int jj = 0; jj < NA; ++jj) {
      const float2 f = ((jj >> bit) & 1) ? wc : w;
      cmul_in(a[jj], f);
      if constexpr (BWD) cmul_in(l[jj], f);
    }
  }
  // Im<lambda|P_q|psi> (P = X, Y, Z) of m register bits: wave sums into LDS
  __device__ __forceinline__ void func(float2 (&a)[NA], float2 (&l)[NA], float2& ph, int m, int first, int) const {
    if constexpr (BWD) {
      // functionals of every register bit; entry j (register bit j) names the
      // run's slot, or -1 when the bit holds no run of this group
      const FuncEntry* fe = A.funcs + first;
      // the slots of the R register bits, read as uniform scalars
      int sl[R];
#pragma unroll
      for (int j = 0; j < R; ++j) sl[j] = cld(&fe[j].slot);
      // part[wave][slot][Pauli], through an LDS-typed pointer
      __attribute__((address_space(3))) float* part = (__attribute__((address_space(3))) float*)qf_pass_part;
      if constexpr (R == 4) {
        float v[12];
        float z[R];
        func_z_all<R>(a, l, z);
#pragma unroll
        for (int j = 0; j < R; ++j) {
          v[3 * j] = v[3 * j + 1] = 0.f;
          v[3 * j + 2] = z[j];
        }
        func_xy_all<R>(a, l, v);
        // lanes beyond a small tile hold copies of in-tile elements: no share
        // (workgroups of more than 64 threads always cover whole tiles)
        if constexpr (NT == 64) {
          if (A.tb < 6 && !active) {
#pragma unroll
            for (int i = 0; i < 12; ++i) v[i] = 0.f;
          }
        }
        const float sum = wave_reduce12(v, lane);
        // the slots of bits 0,1 and 2,3 as 16-bit halves (no run: 0xffff); a
        // lane picks its half with lane bits 5 and 4, which give its register bit
        const uint32_t slots01 = ((uint32_t)sl[0] & 0xffffu) | ((uint32_t)sl[1] << 16);
        const uint32_t slots23 = ((uint32_t)sl[2] & 0xffffu) | ((uint32_t)sl[3] << 16);
        const uint32_t slot = (((lane & 32) ? slots23 : slots01) >> (lane & 16)) & 0xffffu;
        if (wave_sum_writer12(lane) && slot != 0xffffu)
          part[wave * 3 * n_slots + 3 * (int)slot + wave_sum_pauli12(lane)] = sum;
      } else {
        float v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = 0.f;
        func3_all<R>(a, l, v);
        if constexpr (NT == 64) {
          if (A.tb < 6 && !active) {
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = 0.f;
          }
        }
        const float sum = wave_reduce16(v, lane);
        const int idx = wave_sum_index(lane);
        if (wave_sum_writer(lane) && idx < 3 * R) {
          const int e = idx / 3, pq = idx - 3 * e;
          int slot = sl[0];
#pragma unroll
          for (int j = 1; j < R; ++j) slot = (e == j) ? sl[j] : slot;
          if (slot >= 0) part[wave * 3 * n_slots + 3 * slot + pq] = sum;
        }
      }
    }
  }
};

template <int R, int NT, bool BWD>
__device__ __forceinline__ void pass_body(const KArgs& A, const int item) {
  // the tile: a static array, so that its base folds into the LDS offsets
  __shared__ float2 lds[(1 << R) * NT];
  constexpr int NA = 1 << R;
  constexpr int WAVES = NT / 64;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int tb = A.tb;
  const bool active = t < (1 << tb);
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

  const PassCtx<R, NT, BWD> cx{A, lds, t, tlog, active, sample, lane, wave, n_slots};
  // bases of the layout the tile is in (cur_idx: its index, -1 = not loaded)
  int cur_idx = -1;
  uint2 cur = make_uint2(0u, 0u);

  // the next op record is fetched while the current one executes
  Op next = ld_op(A.ops);
  for (int oi = 0; oi < A.n_ops; ++oi) {
    const Op op = next;
    if (oi + 1 < A.n_ops) next = ld_op(A.ops + oi + 1);
    switch (op.kind) {
      case OP_INIT0: {
        const LayoutRec* L = A.layouts + op.a;
        const uint32_t base = cx.log_base(op.a, cur_idx, cur);
        RegBits<R> rb;
        rb.load(L->log_reg);
#pragma unroll
        for (int jj = 0; jj < NA; ++jj)
          a[jj] = make_float2((active && (base | rb(jj)) == 0u) ? 1.f : 0.f, 0.f);
        break;
      }
      case OP_LOAD: {
        const LayoutRec* L = A.layouts + op.a;
        const uint32_t base = (op.c ? tout : tin) | cx.mem_base(op.a);
        RegBits<R> rb;
        rb.load(L->mem_reg);
        // every lane loads: the thread tables are zero above the tile's thread
        // bits, so lanes beyond the tile read (and later drop) in-tile elements;
        // an unpredicated load keeps the register arrays in place
        if (op.b == 0 && A.src0_bf16) {
          const uint32_t* src = reinterpret_cast<const uint32_t*>(A.src0) + (long long)sl * A.s0;
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) a[jj] = widen_bf16x2(src[base | rb(jj)]);
        } else if (op.b == 0) {
          const float2* src = reinterpret_cast<const float2*>(A.src0) + (long long)sl * A.s0;
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) a[jj] = src[base | rb(jj)];
        } else if constexpr (BWD) {
          const float2* src = reinterpret_cast<const float2*>(A.src1) + (long long)sl * A.s1;
#pragma unroll
          for (int jj = 0; jj < NA; ++jj) l[jj] = src[base | rb(jj)];
        }
        break;
      }
      case OP_STORE: {
        // flush the pending phase (an exact identity when none is pending)
        scale_all<NA>(a, ph);
        if constexpr (BWD) scale_all<NA>(l, ph);
        ph = make_float2(1.f, 0.f);
        const LayoutRec* L = A.layouts + op.a;
        const uint32_t base = (op.c ? tout : tin) | cx.mem_base(op.a);
        RegBits<R> rb;
        rb.load(L->mem_reg);
        if (active && A.dst) {
          float2* dst = reinterpret_cast<float2*>(A.dst) + (long long)sl * A.sd;
          if constexpr (BWD) {
            if (A.dpsi) {
              // also psi, un-applied to the pass input, in the same memory order
              float2* dp = reinterpret_cast<float2*>(A.dpsi) + (long long)sl * A.sdp;
#pragma unroll
              for (int jj = 0; jj < NA; ++jj) {
                const uint32_t i = base | rb(jj);
                dst[i] = l[jj];
                dp[i] = a[jj];
              }
            } else {
#pragma unroll
              for (int jj = 0; jj < NA; ++jj) dst[base | rb(jj)] = l[jj];
            }
          } else {
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) dst[base | rb(jj)] = a[jj];
            if (A.dst2) {
              uint32_t* dst2 = A.dst2 + (long long)sl * A.sd2;
#pragma unroll
              for (int jj = 0; jj < NA; ++jj) dst2[base | rb(jj)] = pack_bf16x2(a[jj]);
            }
          }
        }
        break;
      }
      case OP_PERM: {
        const uint32_t bf = op.a == cur_idx ? cur.x : cx.base2(op.a).x;
        cur = cx.base2(op.b);
        cur_idx = op.b;
        cx.perm(a, l, ph, op.a, op.b, bf, cur.x);
        break;
      }
      case OP_RY:
        cx.ry(a, l, ph, op.a, op.b);
        break;
      case OP_RYG:
        cx.ryg(a, l, ph, op.b, op.c);
        break;
      case OP_DIAGT:
        cx.diagt(a, l, ph, cx.log_base(op.a, cur_idx, cur), op.b, op.c, op.d, op.e);
        break;
      case OP_CZA:
        cx.cza(a, l, ph, op.a, cx.log_base(op.b, cur_idx, cur));
        break;
      case OP_PHASEA:
        cx.phasea(a, l, ph, op.a, op.b);
        break;
      case OP_EPOCH: {
        // a run of consecutive register epochs, one iteration each, with the
        // sub-steps of an epoch in program order; every epoch has its PERM and
        // applies its run group (mask 0: identity), so the loop body has one path
        for (int ei = op.a; ei < op.a + op.b; ++ei) {
          const EpochRec* E = A.epochs + ei;
          const int perm_from = cld(&E->perm_from), perm_to = cld(&E->perm_to);
          const int diag_layout = cld(&E->diag_layout);
          const int n_pha = cld(&E->pha_count), pha0 = cld(&E->pha_first);
          const int cza = cld(&E->cza), cza_layout = cld(&E->cza_layout);
          const int ry_first = cld(&E->ry_a), ry_mask = cld(&E->ry_b);
          if constexpr (!BWD) {
            // bases before the PERM: carried from the previous epoch (the planner chains
            // the layouts; the load is a fallback), requested before those after it so
            // that the LDS writes wait for the first load only
            uint32_t bf = cur.x;
            if (perm_from != cur_idx) bf = cx.base2(perm_from).x;
            const uint2 nb = cx.base2(perm_to);
            cx.perm(a, l, ph, perm_from, perm_to, bf, nb.x);
            cur = nb;
            cur_idx = perm_to;
            if (diag_layout >= 0)
              cx.diagt(a, l, ph, cx.log_base(diag_layout, cur_idx, cur), cld(&E->czg_first), cld(&E->czg_count),
                       cld(&E->pev_first), cld(&E->pev_count));
            for (int p = pha0; p < pha0 + n_pha; ++p) cx.phasea(a, l, ph, cld(&A.phas[p].regbit), cld(&A.phas[p].pev));
            if (cza >= 0) cx.cza(a, l, ph, cza, cx.log_base(cza_layout, cur_idx, cur));
            cx.ryg(a, l, ph, ry_first, ry_mask);
          } else {
            // the tile is in layout perm_from until the PERM that ends the epoch
            if (perm_from != cur_idx) {
              cur = cx.base2(perm_from);
              cur_idx = perm_from;
            }
            // bases after the PERM, requested now: the epoch's work hides the load
            const uint2 nb = cx.base2(perm_to);
            const int n_func = cld(&E->func_count);
            if (n_func > 0) cx.func(a, l, ph, n_func, cld(&E->func_first), 0);
            cx.ryg(a, l, ph, ry_first, ry_mask);
            if (cza >= 0) cx.cza(a, l, ph, cza, cx.log_base(cza_layout, cur_idx, cur));
            for (int p = pha0; p < pha0 + n_pha; ++p) cx.phasea(a, l, ph, cld(&A.phas[p].regbit), cld(&A.phas[p].pev));
            if (diag_layout >= 0)
              cx.diagt(a, l, ph, cx.log_base(diag_layout, cur_idx, cur), cld(&E->czg_first), cld(&E->czg_count),
                       cld(&E->pev_first), cld(&E->pev_count));
            cx.perm(a, l, ph, perm_from, perm_to, cur.x, nb.x);
            cur = nb;
            cur_idx = perm_to;
          }
        }
        break;
      }
      case OP_EXPECT: {
        if constexpr (!BWD) {
          if (!A.do_expect) break;
          const LayoutRec* L = A.layouts + op.a;
          const uint32_t base = cx.log_base(op.a, cur_idx, cur);
          RegBits<R> rb;
          rb.load(L->log_reg);
          for (int k0 = 0; k0 < A.K; k0 += 16) {
            float v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = 0.f;
#pragma unroll
            for (int jj = 0; jj < NA; ++jj) {
              const uint32_t x = base | rb(jj);
              // lanes beyond a small tile hold copies of in-tile elements
              const float p = active ? fmaf(a[jj].x, a[jj].x, a[jj].y * a[jj].y) : 0.f;
#pragma unroll
              for (int k = 0; k < 16; ++k)
                if (k0 + k < A.K) v[k] += (__popc(x & cld(A.zmask + k0 + k)) & 1) ? -p : p;
            }
            const float s = wave_reduce16(v, lane);
            const int idx = wave_sum_index(lane);
            if (wave_sum_writer(lane) && k0 + idx < A.K)
              A.partE[((size_t)item * WAVES + wave) * A.K + k0 + idx] = s;
          }
        }
        break;
      }
      case OP_SEED: {
        if constexpr (BWD) {
          const LayoutRec* L = A.layouts + op.a;
          const uint32_t base = cx.log_base(op.a, cur_idx, cur);
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
      case OP_FUNC:
        cx.func(a, l, ph, op.a, op.b, op.c);
        break;
      default:
        break;
    }
  }
  if constexpr (BWD) {
    // one partial sum per tile and functional: add the waves' sums
    if (n_slots > 0) {
      __syncthreads();
      const float* part = qf_pass_part;
      for (int i = t; i < 3 * n_slots; i += NT) {
        float acc = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) acc += part[w * 3 * n_slots + i];
        A.partF[(size_t)item * 3 * n_slots + i] = acc;
      }
    }
  }
}

}  // namespace qf
