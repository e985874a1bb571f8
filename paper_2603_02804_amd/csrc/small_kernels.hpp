// small_kernels.hpp -- device code of the coefficient, gradient-assembly and
// reduction kernels (the 2x2 run algebra in double precision), shared by the
// single-plan kernels, the merged mixed-batch kernels and the complex128
// validation path.
#pragma once
#include <hip/hip_runtime.h>

#include "small_args.hpp"

namespace qf {

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

template <class Real>
__device__ inline double gate_angle(const Tabs& T, const GateRec& g, const Real* theta, const Real* x, int F,
                                    int sample) {
  if (g.theta_idx <= -2) return T.consts[-2 - g.theta_idx];   // fixed angle of an internal gate
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

template <class Real>
__device__ inline D2 run_matrix(const Tabs& T, const RunRec& rr, const Real* theta, const Real* x, int F,
                                int sample) {
  D2 U = d2_eye();
  for (int i = 0; i < rr.gate_count; ++i) {
    const GateRec g = T.gates[T.run_gates[rr.gate_begin + i]];
    U = d2_mul(d2_rot(g.kind, gate_angle(T, g, theta, x, F, sample)), U);
  }
  return U;
}

// Run coefficients.  zyz = 1: [cos(b/2), sin(b/2), u, v, tan(b/4)] of the RZ RY RZ split;
// zyz = 0: the 2x2 matrix row-major (one-gate runs of the per-gate baseline).
template <class Real>
__device__ inline void coef_body(const CoefArgsT<Real>& a, long long idx) {
  if (idx >= a.n_sh + (long long)a.n_ps * a.B) return;
  int r, sample;
  Real* out;
  if (idx < a.n_sh) {
    r = a.T.coef_runs_sh[idx];
    sample = 0;
    out = a.csh + 8 * idx;
  } else {
    const long long j = idx - a.n_sh;
    sample = (int)(j / a.n_ps);
    const int i = (int)(j - (long long)sample * a.n_ps);
    r = a.T.coef_runs_ps[i];
    out = a.cps + 8 * j;
  }
  const D2 U = run_matrix(a.T, a.T.runs[r], a.theta, a.x, a.F, sample);
  if (a.zyz) {
    const ZYZ z = zyz_split(U);
    out[0] = (Real)z.cb; out[1] = (Real)z.sb;
    out[2] = (Real)z.ur; out[3] = (Real)z.ui;
    out[4] = (Real)z.vr; out[5] = (Real)z.vi;
    out[6] = (Real)(z.sb / (1.0 + z.cb));   // tan(f/2) of the rotation by f = b/2, f in [0, pi/2]
    out[7] = 0;
  } else {
    for (int i = 0; i < 4; ++i) {
      out[2 * i] = (Real)U.r[i];
      out[2 * i + 1] = (Real)U.i[i];
    }
  }
}

// Phase event coefficients w = u(prev run) * v(next run).
__device__ inline void event_body(const EventArgs& a, long long idx) {
  if (idx >= a.n_ev_sh + (long long)a.n_ev_ps * a.B) return;
  int sample = 0;
  EventRec e;
  float* out;
  if (idx < a.n_ev_sh) {
    e = a.T.events[idx];
    out = a.esh + 2 * idx;
  } else {
    const long long j = idx - a.n_ev_sh;
    sample = (int)(j / a.n_ev_ps);
    const int i = (int)(j - (long long)sample * a.n_ev_ps);
    e = a.T.events[a.n_ev_sh + i];
    out = a.eps + 2 * j;
  }
  auto row = [&](int ref) {
    return ref >= 0 ? a.csh + 8 * (long long)ref : a.cps + 8 * ((long long)sample * a.n_ps + (-1 - ref));
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
template <class Real>
__device__ inline void run_grads(const Tabs& T, int r, const Real* theta, const Real* x, int F, int sample,
                                 double fx, double fy, double fz, Real* Grow, int zyz) {
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
    Grow[g.out_idx] = (Real)(0.5 * (gr * fx + gi * fy + G.r[0] * fz));
    K = d2_mul(K, d2_rot(g.kind, gate_angle(T, g, theta, x, F, sample)));
  }
}

// One block per (sample, pass of the segment): sum the pass's per-tile

// One block per (sample, pass of the segment): sum the pass's per-tile
// functional partials (coalesced over the slots), then one thread per run turns
// the three sums into the run's per-gate gradients.  fsum: 3 * max_slots doubles
// of LDS.
__device__ inline void assemble_body(const AssembleArgs& a, int blk, double* fsum) {
  const int s = blk / a.np, p = a.p0 + (blk - s * a.np);
  const int ns = a.T.passes[p].n_slots;
  if (ns == 0) return;
  const float* base = a.partF + (long long)a.nb * a.T.partF_off[p] + (long long)s * a.tiles * 3 * ns;
  for (int v = threadIdx.x; v < 3 * ns; v += blockDim.x) {
    double acc = 0;
    for (int tile = 0; tile < a.tiles; ++tile) acc += base[(long long)tile * 3 * ns + v];
    fsum[v] = acc;
  }
  __syncthreads();
  const int rb = a.T.pass_run_begin[p];
  for (int i = threadIdx.x; i < ns; i += blockDim.x)
    run_grads(a.T, a.T.pass_runs[rb + i], a.theta, a.x, a.F, a.sample0 + s, fsum[3 * i], fsum[3 * i + 1],
              fsum[3 * i + 2], a.Gr + (long long)s * a.n_angle, 1);
}

// theta: sum over the micro-batch and over the gates sharing the angle; x: sum
// over the gates sharing the input, per sample.  Block blk < th_blocks owns
// angles [blk * cols, (blk + 1) * cols): thread t takes angle t % cols and sample
// lane t / cols, sums its samples (lane, lane + lanes, ...) in order, and the
// lanes are added by a fixed pairwise tree in LDS (red: kSmallThreads doubles), so
// the result does not depend on scheduling.  The later blocks form dx, one thread
// per (sample, input).
template <class Real>
__device__ inline void reduce_grads_body(const ReduceGArgsT<Real>& a, int blk, int t, double* red) {
  if (blk < a.th_blocks) {
    const int cols = a.cols, lanes = kSmallThreads / cols;
    const int col = t % cols, lane = t / cols;
    const int p = blk * cols + col;
    double acc = 0;
    if (p < a.P) {
      const int r0 = a.T.th_ref_begin[p], r1 = a.T.th_ref_begin[p + 1];
      for (int s = lane; s < a.nb; s += lanes)
        for (int i = r0; i < r1; ++i) acc += a.Gr[(long long)s * a.n_angle + a.T.th_refs[i]];
    }
    red[t] = acc;
    __syncthreads();
    for (int half = lanes / 2; half >= 1; half /= 2) {
      if (lane < half) red[t] += red[t + half * cols];
      __syncthreads();
    }
    if (lane == 0 && p < a.P) {
      const double sum = red[col];
      a.dtheta[p] = a.accumulate ? a.dtheta[p] + (Real)sum : (Real)sum;
    }
    return;
  }
  const long long j = (long long)(blk - a.th_blocks) * kSmallThreads + t;
  if (!a.dx || j >= (long long)a.nb * a.F) return;
  const int s = (int)(j / a.F), f = (int)(j - (long long)s * a.F);
  double acc = 0;
  for (int i = a.T.in_ref_begin[f]; i < a.T.in_ref_begin[f + 1]; ++i)
    acc += a.Gr[(long long)s * a.n_angle + a.T.in_refs[i]];
  a.dx[(long long)(a.sample0 + s) * a.F + f] = (Real)acc;
}

template <class Real>
__device__ inline void reduce_E_body(const ReduceEArgsT<Real>& a, long long idx) {
  if (idx >= (long long)a.nb * a.K) return;
  const int s = (int)(idx / a.K), k = (int)(idx - (long long)s * a.K);
  double acc = 0;
  for (int i = 0; i < a.parts; ++i) acc += a.partE[((long long)s * a.parts + i) * a.K + k];
  a.E[(long long)(a.sample0 + s) * a.K + k] = (Real)acc;
}

}  // namespace qf
