// plancheck.cpp -- CPU execution of fused pass programs, for testing the planner.
//
// TEST-ONLY.  Built into libqfuse_plancheck.so, which the product library never
// links or loads.  It runs the planner's op programs with the same per-lane
// register / LDS / address-table semantics as the pass kernels, one emulated
// thread at a time, so that schedules, layouts, memory maps and the driver's
// segment and micro-batch sequencing can be checked against the oracle without a
// GPU.  It is not a fallback: the device entry points never reach this code.
#include <cmath>
#include <complex>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include <memory>

#include "batch.hpp"
#include "driver.hpp"

namespace qf {
namespace {

// bfloat16 storage of the memory-saving mode: round to nearest even (NaN kept
// quiet) and the exact widening.
inline uint16_t bf16_round(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
inline float bf16_widen(uint16_t h) {
  const uint32_t u = uint32_t(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

using cd = std::complex<double>;

struct M2 {
  cd m[4];
};

M2 mul(const M2& a, const M2& b) {
  M2 r;
  r.m[0] = a.m[0] * b.m[0] + a.m[1] * b.m[2];
  r.m[1] = a.m[0] * b.m[1] + a.m[1] * b.m[3];
  r.m[2] = a.m[2] * b.m[0] + a.m[3] * b.m[2];
  r.m[3] = a.m[2] * b.m[1] + a.m[3] * b.m[3];
  return r;
}

M2 rot(int kind, double phi) {
  const double c = std::cos(0.5 * phi), s = std::sin(0.5 * phi);
  M2 u;
  if (kind == QF_RX) { u.m[0] = c; u.m[1] = cd(0, -s); u.m[2] = cd(0, -s); u.m[3] = c; }
  else if (kind == QF_RY) { u.m[0] = c; u.m[1] = -s; u.m[2] = s; u.m[3] = c; }
  else { u.m[0] = cd(c, -s); u.m[1] = 0; u.m[2] = 0; u.m[3] = cd(c, s); }
  return u;
}

M2 pauli(int kind) {
  M2 p;
  if (kind == QF_RX) { p.m[0] = 0; p.m[1] = 1; p.m[2] = 1; p.m[3] = 0; }
  else if (kind == QF_RY) { p.m[0] = 0; p.m[1] = cd(0, -1); p.m[2] = cd(0, 1); p.m[3] = 0; }
  else { p.m[0] = 1; p.m[1] = 0; p.m[2] = 0; p.m[3] = -1; }
  return p;
}

M2 dag(const M2& a) {
  M2 r;
  r.m[0] = std::conj(a.m[0]);
  r.m[1] = std::conj(a.m[2]);
  r.m[2] = std::conj(a.m[1]);
  r.m[3] = std::conj(a.m[3]);
  return r;
}

struct CF {
  float re, im;
};
using cf = std::complex<float>;

inline CF cmul(float ar, float ai, CF b) { return {ar * b.re - ai * b.im, ar * b.im + ai * b.re}; }

[[noreturn]] void oob(const char* what) { throw std::runtime_error(std::string("out of bounds: ") + what); }

struct CpuExec {
  const PlanCore& c;
  const char* ws_lo = nullptr;   // workspace range every state / partial access must stay in
  const char* ws_hi = nullptr;
  const char* in_lo = nullptr;   // caller's initial states: the other range reads may use
  const char* in_hi = nullptr;
  void in_ws(const void* p, size_t bytes, const char* what) const {
    const char* q = (const char*)p;
    if (in_lo && q >= in_lo && q + bytes <= in_hi) return;
    if (ws_lo && (q < ws_lo || q + bytes > ws_hi)) oob(what);
  }
  const float* theta = nullptr;
  const float* x = nullptr;
  const float* coef_sh = nullptr;
  const float* coef_ps = nullptr;
  explicit CpuExec(const PlanCore& pc) : c(pc) {}

  qf_status status() const { return QF_OK; }

  double angle(const GateRec& g, int sample) const {
    if (g.theta_idx <= -2) return c.C.consts[-2 - g.theta_idx];
    return g.theta_idx >= 0 ? (double)theta[g.theta_idx] : (double)x[(int64_t)sample * c.C.F + g.input_idx];
  }
  M2 run_matrix(int r, int sample) const {
    const RunRec& rr = c.S.runs[r];
    M2 U;
    U.m[0] = 1; U.m[1] = 0; U.m[2] = 0; U.m[3] = 1;
    for (int i = 0; i < rr.gate_count; ++i) {
      const GateRec& g = c.S.gates[c.S.run_gates[rr.gate_begin + i]];
      U = mul(rot(g.kind, angle(g, sample)), U);
    }
    return U;
  }
  static void put(float* dst, const M2& U) {
    for (int i = 0; i < 4; ++i) {
      dst[2 * i] = (float)U.m[i].real();
      dst[2 * i + 1] = (float)U.m[i].imag();
    }
  }

  const float* ev_sh = nullptr;
  const float* ev_ps = nullptr;

  // RZ(a) RY(b) RZ(c) split: (cos b/2, sin b/2, e^{-ia/2}, e^{-ic/2}) and e^{-ia}.
  struct Split {
    double cb, sb;
    cd u, v, z;
  };
  static Split split(const M2& V) {
    Split o;
    const double a0 = std::abs(V.m[0]), b0 = std::abs(V.m[2]);
    const double nrm = std::sqrt(a0 * a0 + b0 * b0);
    o.cb = a0 / nrm;
    o.sb = b0 / nrm;
    const cd A = a0 > 1e-300 ? V.m[0] / a0 : cd(1, 0);
    const cd Bp = b0 > 1e-300 ? V.m[2] / b0 : cd(1, 0);
    o.z = A * std::conj(Bp);
    o.u = std::polar(1.0, 0.5 * std::arg(o.z));
    o.v = A * std::conj(o.u);
    return o;
  }

  void coef(const float* th, const float* xx, char* ws) {
    theta = th;
    x = xx;
    float* csh = at<float>(ws, c.off_coef_sh);
    float* cps = at<float>(ws, c.off_coef_ps);
    float* esh = at<float>(ws, c.off_ev_sh);
    float* eps = at<float>(ws, c.off_ev_ps);
    coef_sh = csh;
    coef_ps = cps;
    ev_sh = esh;
    ev_ps = eps;
    auto put_run = [&](float* dst, int r, int b) {
      const M2 U = run_matrix(r, b);
      if (c.per_gate) {
        put(dst, U);
        return;
      }
      const Split z = split(U);
      const float v[8] = {(float)z.cb, (float)z.sb, (float)z.u.real(), (float)z.u.imag(),
                          (float)z.v.real(), (float)z.v.imag(), (float)(z.sb / (1.0 + z.cb)), 0.f};
      std::memcpy(dst, v, sizeof(v));
    };
    for (size_t i = 0; i < c.coef_runs_sh.size(); ++i) put_run(csh + 8 * i, c.coef_runs_sh[i], 0);
    const int nps = (int)c.coef_runs_ps.size();
    for (int b = 0; b < c.B; ++b)
      for (int i = 0; i < nps; ++i) put_run(cps + 8 * ((int64_t)b * nps + i), c.coef_runs_ps[i], b);
    auto ev = [&](const EventRec& e, int b, float* out) {
      cf w(1.f, 0.f);
      if (e.prev_ref != INT32_MIN) {
        const float* p = coef_row(e.prev_ref, b);
        w = w * cf(p[2], p[3]);
      }
      if (e.next_ref != INT32_MIN) {
        const float* p = coef_row(e.next_ref, b);
        w = w * cf(p[4], p[5]);
      }
      out[0] = w.real();
      out[1] = w.imag();
    };
    for (int i = 0; i < c.S.n_ev_shared; ++i) ev(c.S.events[i], 0, esh + 2 * i);
    for (int b = 0; b < c.B; ++b)
      for (int i = 0; i < c.S.n_ev_ps; ++i)
        ev(c.S.events[c.S.n_ev_shared + i], b, eps + 2 * ((int64_t)b * c.S.n_ev_ps + i));
  }

  cf event_w(int ref, int sample) const {
    const float* p = ref >= 0 ? ev_sh + 2 * ref : ev_ps + 2 * ((int64_t)sample * c.S.n_ev_ps + (-1 - ref));
    return cf(p[0], p[1]);
  }

  const float* coef_row(int ref, int sample) const {
    if (ref >= 0) return coef_sh + 8 * ref;
    return coef_ps + 8 * ((int64_t)sample * c.S.n_coef_ps + (-1 - ref));
  }

  // ---------------------------------------------------------------- fused pass
  void pass(const PassLaunch& L) {
    const Schedule& S = c.S;
    const PassRec& pr = S.passes[L.pass];
    const int R = S.R, NA = 1 << R, tb = S.thread_bits, active = S.active;
    const int tiles = c.tiles, waves = c.waves, K = c.C.K;
    const int b0 = L.bwd ? pr.bop_begin : (L.load_input ? pr.fload_begin : pr.fop_begin);
    const int nops = L.bwd ? pr.bop_count : pr.fop_count;
    const int64_t k_amps = int64_t(1) << S.k;
    std::vector<CF> a(size_t(active) * NA), l(size_t(active) * NA), lds(k_amps);
    for (int sl = 0; sl < L.nb; ++sl) {
      const int sample = L.sample0 + sl;
      for (int tile = 0; tile < tiles; ++tile) {
        uint32_t tlog = 0, tin = 0, tout = 0;
        for (int i = 0; i < pr.n_nonlocal; ++i)
          if ((tile >> i) & 1) {
            tlog |= 1u << pr.nl_log[i];
            tin |= 1u << pr.nl_in[i];
            tout |= 1u << pr.nl_out[i];
          }
        std::fill(a.begin(), a.end(), CF{0, 0});
        std::fill(l.begin(), l.end(), CF{0, 0});
        std::vector<cf> ph(active, cf(1.f, 0.f));   // pending per-thread phase
        auto flush = [&]() {
          for (int t = 0; t < active; ++t) {
            for (int jj = 0; jj < NA; ++jj) {
              cf v = cf(a[t * NA + jj].re, a[t * NA + jj].im) * ph[t];
              a[t * NA + jj] = CF{v.real(), v.imag()};
              if (L.bwd) {
                cf w = cf(l[t * NA + jj].re, l[t * NA + jj].im) * ph[t];
                l[t * NA + jj] = CF{w.real(), w.imag()};
              }
            }
            ph[t] = cf(1.f, 0.f);
          }
        };
        auto tbase = [&](const uint32_t* tab, int t) {
          uint32_t v = 0;
          for (int i = 0; i < tb; ++i)
            if ((t >> i) & 1) v ^= tab[i];
          return v;
        };
        const int64_t item = (int64_t)sl * tiles + tile;
        for (int oi = 0; oi < nops; ++oi) {
          const std::vector<Op> seq = expand_op(S.ops[b0 + oi], L.bwd);
          for (const Op& op : seq) {
          switch (op.kind) {
            case OP_INIT0: {
              const LayoutRec& Ly = S.layouts[op.a];
              for (int t = 0; t < active; ++t)
                for (int jj = 0; jj < NA; ++jj) {
                  uint32_t xl = tlog | tbase(Ly.log_thr, t) | reg_index(Ly.log_reg, jj);
                  a[t * NA + jj] = (xl == 0) ? CF{1, 0} : CF{0, 0};
                }
              break;
            }
            case OP_LOAD: {
              const LayoutRec& Ly = S.layouts[op.a];
              const float* src = op.b == 0 ? L.src0 : L.src1;
              const int64_t stride = op.b == 0 ? L.src0_stride : L.src1_stride;
              std::vector<CF>& v = op.b == 0 ? a : l;
              const uint32_t tm = op.c ? tout : tin;
              const bool bf = op.b == 0 && L.src0_bf16;
              for (int t = 0; t < active; ++t)
                for (int jj = 0; jj < NA; ++jj) {
                  uint64_t idx = tm | tbase(Ly.mem_thr, t) | reg_index(Ly.mem_reg, jj);
                  if (idx >= (uint64_t)c.amps) oob("load index");
                  if (bf) {
                    const uint32_t* p = reinterpret_cast<const uint32_t*>(src) + sl * stride + idx;
                    in_ws(p, 4, "load address");
                    v[t * NA + jj] = CF{bf16_widen(uint16_t(*p & 0xffffu)), bf16_widen(uint16_t(*p >> 16))};
                  } else {
                    const float* p = src + sl * stride + 2 * idx;
                    in_ws(p, 8, "load address");
                    v[t * NA + jj] = CF{p[0], p[1]};
                  }
                }
              break;
            }
            case OP_STORE: {
              flush();
              const LayoutRec& Ly = S.layouts[op.a];
              const std::vector<CF>& v = L.bwd ? l : a;
              const uint32_t tm = op.c ? tout : tin;
              if (!L.dst) break;
              for (int t = 0; t < active; ++t)
                for (int jj = 0; jj < NA; ++jj) {
                  uint64_t idx = tm | tbase(Ly.mem_thr, t) | reg_index(Ly.mem_reg, jj);
                  if (idx >= (uint64_t)c.amps) oob("store index");
                  if (!L.bwd && L.dst2) {
                    uint32_t* q = L.dst2 + sl * L.dst2_stride + idx;
                    in_ws(q, 4, "store address");
                    *q = uint32_t(bf16_round(v[t * NA + jj].re)) | (uint32_t(bf16_round(v[t * NA + jj].im)) << 16);
                  }
                  float* p = L.dst + sl * L.dst_stride + 2 * idx;
                  in_ws(p, 8, "store address");
                  p[0] = v[t * NA + jj].re;
                  p[1] = v[t * NA + jj].im;
                  if (L.bwd && L.dpsi) {   // psi at the pass input (uncompute mode)
                    float* q = L.dpsi + sl * L.dpsi_stride + 2 * idx;
                    in_ws(q, 8, "store address");
                    q[0] = a[t * NA + jj].re;
                    q[1] = a[t * NA + jj].im;
                  }
                }
              break;
            }
            case OP_PERM: {
              flush();
              const LayoutRec& F = S.layouts[op.a];
              const LayoutRec& T = S.layouts[op.b];
              for (int which = 0; which < (L.bwd ? 2 : 1); ++which) {
                std::vector<CF>& v = which == 0 ? a : l;
                std::vector<char> seen(k_amps, 0);
                for (int t = 0; t < active; ++t)
                  for (int jj = 0; jj < NA; ++jj) {
                    uint32_t e = (tbase(F.lds_thr, t) ^ reg_index(F.lds_reg, jj)) / kLdsElemBytes;
                    if (e >= k_amps || seen[e]) throw std::runtime_error("LDS layout is not a bijection");
                    seen[e] = 1;
                    lds[e] = v[t * NA + jj];
                  }
                for (int t = 0; t < active; ++t)
                  for (int jj = 0; jj < NA; ++jj) {
                    uint32_t e = (tbase(T.lds_thr, t) ^ reg_index(T.lds_reg, jj)) / kLdsElemBytes;
                    if (e >= k_amps) oob("LDS read");
                    v[t * NA + jj] = lds[e];
                  }
              }
              break;
            }
            case OP_RY:
            case OP_RYG: {
              const int m = op.kind == OP_RY ? 1 : op.a;
              uint32_t seen = 0;
              for (int e = 0; e < m; ++e) {
                int j = op.a, ref = op.b;
                if (op.kind == OP_RYG) {
                  if (op.b + e >= (int)S.rygs.size()) oob("RYG entry");
                  j = S.rygs[op.b + e].regbit;
                  ref = S.rygs[op.b + e].ref;
                  if (j < 0 || j >= R || ((seen >> j) & 1)) oob("RYG register bit");
                  seen |= 1u << j;
                }
                // rotation by f = b/2 as three shears: tan(f/2) and sin f
                const float* u = coef_row(ref, sample);
                const float tt = L.bwd ? -u[6] : u[6], ss = L.bwd ? -u[1] : u[1];
                for (int which = 0; which < (L.bwd ? 2 : 1); ++which) {
                  std::vector<CF>& v = which == 0 ? a : l;
                  for (int t = 0; t < active; ++t)
                    for (int jj = 0; jj < NA; ++jj) {
                      if ((jj >> j) & 1) continue;
                      CF& x0 = v[t * NA + jj];
                      CF& x1 = v[t * NA + (jj | (1 << j))];
                      x0.re = std::fma(-tt, x1.re, x0.re);
                      x0.im = std::fma(-tt, x1.im, x0.im);
                      x1.re = std::fma(ss, x0.re, x1.re);
                      x1.im = std::fma(ss, x0.im, x1.im);
                      x0.re = std::fma(-tt, x1.re, x0.re);
                      x0.im = std::fma(-tt, x1.im, x0.im);
                    }
                }
              }
              if (op.kind == OP_RYG && (int)seen != op.c) oob("RYG bit mask");
              break;
            }
            case OP_DIAGT: {
              const LayoutRec& Ly = S.layouts[op.a];
              for (int t = 0; t < active; ++t) {
                const uint32_t xl = tlog | tbase(Ly.log_thr, t);
                uint32_t par = 0;
                for (int gi = 0; gi < op.c; ++gi) {
                  const CzGroup& g = S.czg[op.b + gi];
                  par ^= xl & (xl >> g.shift) & g.mask;
                }
                if (__builtin_popcount(par) & 1) ph[t] = -ph[t];
                for (int ei = 0; ei < op.e; ++ei) {
                  const PhaseEv& e = S.pev[op.d + ei];
                  cf w = event_w(e.ref, sample);
                  const bool bit = (xl >> e.q) & 1;
                  if (bit != L.bwd) w = std::conj(w);
                  ph[t] *= w;
                }
              }
              break;
            }
            case OP_CZA: {
              const CzaRec& cr = S.cza[op.a];
              const LayoutRec& Ly = S.layouts[op.b];
              for (int t = 0; t < active; ++t) {
                const uint32_t xl = tlog | tbase(Ly.log_thr, t);
                for (int jj = 0; jj < NA; ++jj) {
                  int sgn = (cr.sr >> jj) & 1;
                  for (int j = 0; j < R; ++j)
                    if ((jj >> j) & 1) sgn ^= __builtin_popcount(xl & cr.cmask[j]) & 1;
                  if (!sgn) continue;
                  a[t * NA + jj] = CF{-a[t * NA + jj].re, -a[t * NA + jj].im};
                  if (L.bwd) l[t * NA + jj] = CF{-l[t * NA + jj].re, -l[t * NA + jj].im};
                }
              }
              break;
            }
            case OP_PHASEA: {
              const PhaseEv& e = S.pev[op.b];
              cf w = event_w(e.ref, sample);
              if (L.bwd) w = std::conj(w);
              for (int which = 0; which < (L.bwd ? 2 : 1); ++which) {
                std::vector<CF>& v = which == 0 ? a : l;
                for (int t = 0; t < active; ++t)
                  for (int jj = 0; jj < NA; ++jj) {
                    const cf f = ((jj >> op.a) & 1) ? std::conj(w) : w;
                    cf y = cf(v[t * NA + jj].re, v[t * NA + jj].im) * f;
                    v[t * NA + jj] = CF{y.real(), y.imag()};
                  }
              }
              break;
            }
            case OP_EXPECT: {
              if (!L.do_expect) break;
              const LayoutRec& Ly = S.layouts[op.a];
              for (int w = 0; w < waves; ++w)
                for (int k = 0; k < K; ++k) {
                  float acc = 0;
                  for (int t = w * 64; t < std::min(active, (w + 1) * 64); ++t)
                    for (int jj = 0; jj < NA; ++jj) {
                      uint32_t xl = tlog | tbase(Ly.log_thr, t) | reg_index(Ly.log_reg, jj);
                      CF v = a[t * NA + jj];
                      float p = v.re * v.re + v.im * v.im;
                      acc += (__builtin_popcount(xl & (uint32_t)c.C.obs[k].z_mask) & 1) ? -p : p;
                    }
                  const int64_t pe = (item * waves + w) * K + k;
                  if (pe >= (int64_t)L.nb * tiles * waves * K) oob("partE");
                  in_ws(L.partE + pe, 4, "partE address");
                  L.partE[pe] = acc;
                }
              break;
            }
            case OP_SEED: {
              const LayoutRec& Ly = S.layouts[op.a];
              for (int t = 0; t < active; ++t)
                for (int jj = 0; jj < NA; ++jj) {
                  uint32_t xl = tlog | tbase(Ly.log_thr, t) | reg_index(Ly.log_reg, jj);
                  float cc = 0;
                  for (int k = 0; k < K; ++k) {
                    float g = L.dE[(int64_t)sample * K + k];
                    cc += (__builtin_popcount(xl & (uint32_t)c.C.obs[k].z_mask) & 1) ? -g : g;
                  }
                  CF v = a[t * NA + jj];
                  l[t * NA + jj] = CF{2 * cc * v.re, 2 * cc * v.im};
                }
              break;
            }
            case OP_FUNC: {
              const int ns = pr.n_slots;
              for (int e = 0; e < op.a; ++e) {
                const FuncEntry& fe = S.funcs[op.b + e];
                if (fe.slot < 0) continue;   // register bit without a run of this group
                const int j = fe.regbit;
                float fw[3] = {0, 0, 0};
                for (int w = 0; w < waves; ++w) {
                  float fx = 0, fy = 0, fz = 0;
                  for (int t = w * 64; t < std::min(active, (w + 1) * 64); ++t)
                    for (int jj = 0; jj < NA; ++jj) {
                      if ((jj >> j) & 1) continue;
                      CF p0 = a[t * NA + jj], p1 = a[t * NA + (jj | (1 << j))];
                      CF l0 = l[t * NA + jj], l1 = l[t * NA + (jj | (1 << j))];
                      fx += l0.re * p1.im - l0.im * p1.re + l1.re * p0.im - l1.im * p0.re;
                      fy += -(l0.re * p1.re + l0.im * p1.im) + (l1.re * p0.re + l1.im * p0.im);
                      fz += (l0.re * p0.im - l0.im * p0.re) - (l1.re * p1.im - l1.im * p1.re);
                    }
                  fw[0] += fx;
                  fw[1] += fy;
                  fw[2] += fz;
                }
                const int64_t pf = item * 3 * ns + 3 * fe.slot;
                if (fe.slot < 0 || fe.slot >= ns || pf + 3 > (int64_t)L.nb * tiles * 3 * ns) oob("partF");
                float* dst = L.partF + pf;
                in_ws(dst, 12, "partF address");
                dst[0] = fw[0];
                dst[1] = fw[1];
                dst[2] = fw[2];
              }
              break;
            }
            default:
              throw std::runtime_error("unknown op");
          }
          }
        }
      }
    }
  }

  // An epoch op as the sub-ops of its epochs in execution order; any other op
  // as itself.
  std::vector<Op> expand_op(const Op& o, bool bwd) const {
    if (o.kind != OP_EPOCH) return {o};
    const Schedule& S = c.S;
    std::vector<Op> out;
    if (o.b < 1 || o.a < 0 || o.a + o.b > (int)S.epochs.size()) oob("epoch records");
    for (int ei = o.a; ei < o.a + o.b; ++ei) {
      const EpochRec& e = S.epochs[ei];
      std::vector<Op> perm, diag, pha, cza, ry, func;
      if (e.perm_from >= 0) perm.push_back({OP_PERM, e.perm_from, e.perm_to, 0, 0, 0, 0, 0});
      if (e.diag_layout >= 0)
        diag.push_back({OP_DIAGT, e.diag_layout, e.czg_first, e.czg_count, e.pev_first, e.pev_count, 0, 0});
      for (int i = 0; i < e.pha_count; ++i) {
        if (e.pha_first + i >= (int)S.phas.size()) oob("epoch PHASEA entry");
        pha.push_back({OP_PHASEA, S.phas[e.pha_first + i].regbit, S.phas[e.pha_first + i].pev, 0, 0, 0, 0, 0});
      }
      if (e.cza >= 0) cza.push_back({OP_CZA, e.cza, e.cza_layout, 0, 0, 0, 0, 0});
      if (e.ry_b != 0) {
        int cnt = 0;
        for (int j = 0; j < 32; ++j) cnt += (e.ry_b >> j) & 1;
        ry.push_back({OP_RYG, cnt, e.ry_a, e.ry_b, 0, 0, 0, 0});
      }
      if (e.func_count > 0) func.push_back({OP_FUNC, e.func_count, e.func_first, 0, 0, 0, 0, 0});
      auto add = [&](const std::vector<Op>& v) { out.insert(out.end(), v.begin(), v.end()); };
      if (!bwd) { add(perm); add(diag); add(pha); add(cza); add(ry); }
      else { add(func); add(ry); add(cza); add(pha); add(diag); add(perm); }
    }
    return out;
  }

  void reduce_E(int nb, int sample0, const float* partE, float* E) {
    const int K = c.C.K;
    for (int s = 0; s < nb; ++s)
      for (int k = 0; k < K; ++k) {
        double acc = 0;
        for (int i = 0; i < c.tiles * c.waves; ++i) acc += partE[((int64_t)s * c.tiles * c.waves + i) * K + k];
        E[(int64_t)(sample0 + s) * K + k] = (float)acc;
      }
  }

  // grad_i = 1/2 Im<lambda| K_i P_i K_i^dag |psi> at the cut after the run,
  // K_i = product of the run's gates after gate i.
  void run_grads(int r, int sample, double fx, double fy, double fz, float* Grow, bool zyz) const {
    const RunRec& rr = c.S.runs[r];
    const cd z = zyz ? split(run_matrix(r, sample)).z : cd(1, 0);
    M2 Kc;
    Kc.m[0] = 1; Kc.m[1] = 0; Kc.m[2] = 0; Kc.m[3] = 1;
    for (int i = rr.gate_count - 1; i >= 0; --i) {
      const GateRec& g = c.S.gates[c.S.run_gates[rr.gate_begin + i]];
      M2 G = mul(mul(Kc, pauli(g.kind)), dag(Kc));
      const cd g10 = z * G.m[2];
      double gr = 0.5 * (g10.real() * fx + g10.imag() * fy + G.m[0].real() * fz);
      Grow[g.out_idx] = (float)gr;
      Kc = mul(Kc, rot(g.kind, angle(g, sample)));
    }
  }

  void assemble(int seg, int nb, int sample0, const float*, const float*, const float* partF, float* Gr) {
    for (int s = 0; s < nb; ++s)
      for (int i = c.seg_run_begin[seg]; i < c.seg_run_begin[seg + 1]; ++i) {
        const int r = c.seg_runs[i];
        const RunRec& rr = c.S.runs[r];
        const int ns = c.S.passes[rr.pass].n_slots;
        const float* base = partF + (int64_t)nb * c.partF_off[rr.pass];
        double f[3] = {0, 0, 0};
        for (int it = 0; it < c.tiles; ++it)
          for (int P = 0; P < 3; ++P) f[P] += base[(((int64_t)s * c.tiles) + it) * 3 * ns + 3 * rr.slot + P];
        run_grads(r, sample0 + s, f[0], f[1], f[2], Gr + (int64_t)s * c.n_angle, true);
      }
  }

  void reduce_grads(int nb, int sample0, const float* Gr, float* dtheta, float* dx, bool accumulate) {
    for (int p = 0; p < c.C.P; ++p) {
      double acc = 0;
      for (int s = 0; s < nb; ++s)
        for (int i = c.th_ref_begin[p]; i < c.th_ref_begin[p + 1]; ++i) acc += Gr[(int64_t)s * c.n_angle + c.th_refs[i]];
      dtheta[p] = accumulate ? dtheta[p] + (float)acc : (float)acc;
    }
    if (dx)
      for (int s = 0; s < nb; ++s)
        for (int f = 0; f < c.C.F; ++f) {
          double acc = 0;
          for (int i = c.in_ref_begin[f]; i < c.in_ref_begin[f + 1]; ++i) acc += Gr[(int64_t)s * c.n_angle + c.in_refs[i]];
          dx[(int64_t)(sample0 + s) * c.C.F + f] = (float)acc;
        }
  }

  // ---------------------------------------------------------------- per-gate baseline
  void pg_coef(const float* th, const float* xx, char* ws) { coef(th, xx, ws); }
  void pg_reduce_grads(int nb, int sample0, const float* Gr, float* dtheta, float* dx, bool accumulate) {
    reduce_grads(nb, sample0, Gr, dtheta, dx, accumulate);
  }
  void pg_init(float* psi, int nb) {
    for (int s = 0; s < nb; ++s) {
      std::memset(psi + s * 2 * c.amps, 0, sizeof(float) * 2 * c.amps);
      psi[s * 2 * c.amps] = 1;
    }
  }
  void pg_copy(float* dst, const float* src, int nb) { std::memcpy(dst, src, sizeof(float) * 2 * c.amps * nb); }
  void apply1(float* v, int q, const float* u) {
    const int64_t st = int64_t(1) << q;
    for (int64_t i = 0; i < c.amps; ++i) {
      if (i & st) continue;
      CF x0{v[2 * i], v[2 * i + 1]}, x1{v[2 * (i | st)], v[2 * (i | st) + 1]};
      CF p = cmul(u[0], u[1], x0), q2 = cmul(u[2], u[3], x1);
      CF r = cmul(u[4], u[5], x0), s2 = cmul(u[6], u[7], x1);
      v[2 * i] = p.re + q2.re; v[2 * i + 1] = p.im + q2.im;
      v[2 * (i | st)] = r.re + s2.re; v[2 * (i | st) + 1] = r.im + s2.im;
    }
  }
  void pg_rot(float* psi, int nb, int sample0, int r, const float*, const float*) {
    for (int s = 0; s < nb; ++s) apply1(psi + s * 2 * c.amps, c.S.runs[r].q, coef_row(c.S.runs[r].coef, sample0 + s));
  }
  void pg_cz(float* psi, float* lam, int nb, int qa, int qb) {
    for (int s = 0; s < nb; ++s)
      for (int64_t i = 0; i < c.amps; ++i)
        if (((i >> qa) & 1) && ((i >> qb) & 1)) {
          for (int w = 0; w < 2; ++w) {
            float* v = (w == 0 ? psi : lam);
            if (!v) continue;
            v[s * 2 * c.amps + 2 * i] *= -1;
            v[s * 2 * c.amps + 2 * i + 1] *= -1;
          }
        }
  }
  // observables (any Pauli strings, masks in the stored state's bit order);
  // strides count floats
  void pauli_expect(const float* psi, int64_t stride, int nb, float* partE) {
    const std::vector<PauliRec> ob = pauli_table(c);
    for (int s = 0; s < nb; ++s)
      for (int k = 0; k < c.C.K; ++k) {
        const PauliRec& o = ob[k];
        double acc = 0;
        for (int64_t y = 0; y < c.amps; ++y) {
          const int64_t yx = y ^ (int64_t)o.xm;
          in_ws(psi + s * stride + 2 * y, 8, "expect address");
          const double ar = psi[s * stride + 2 * y], ai = psi[s * stride + 2 * y + 1];
          const double br = psi[s * stride + 2 * yx], bi = psi[s * stride + 2 * yx + 1];
          double cr = ar * br + ai * bi, ci = ar * bi - ai * br;   // conj(a) b
          for (int t = 0; t < o.ny; ++t) { const double tr = -ci; ci = cr; cr = tr; }
          acc += (__builtin_popcountll((uint64_t)(yx & (int64_t)o.zm)) & 1) ? -cr : cr;
        }
        for (int b = 0; b < c.pauli_blocks; ++b)
          partE[((int64_t)s * c.pauli_blocks + b) * c.C.K + k] = b == 0 ? (float)acc : 0.f;
      }
  }
  void pauli_reduce_E(int nb, int sample0, const float* partE, float* E) {
    for (int s = 0; s < nb; ++s)
      for (int k = 0; k < c.C.K; ++k) {
        double acc = 0;
        for (int b = 0; b < c.pauli_blocks; ++b) acc += partE[((int64_t)s * c.pauli_blocks + b) * c.C.K + k];
        E[(int64_t)(sample0 + s) * c.C.K + k] = (float)acc;
      }
  }
  void pauli_seed(const float* psi, int64_t ps, float* lam, int64_t ls, int nb, int sample0, const float* dE) {
    const std::vector<PauliRec> ob = pauli_table(c);
    for (int s = 0; s < nb; ++s)
      for (int64_t y = 0; y < c.amps; ++y) {
        double ar = 0, ai = 0;
        for (int k = 0; k < c.C.K; ++k) {
          const PauliRec& o = ob[k];
          const int64_t yx = y ^ (int64_t)o.xm;
          double g = dE[(int64_t)(sample0 + s) * c.C.K + k];
          if (__builtin_popcountll((uint64_t)(yx & (int64_t)o.zm)) & 1) g = -g;
          double tr = psi[s * ps + 2 * yx], ti = psi[s * ps + 2 * yx + 1];
          for (int t = 0; t < o.ny; ++t) { const double u = -ti; ti = tr; tr = u; }
          ar += g * tr;
          ai += g * ti;
        }
        in_ws(lam + s * ls + 2 * y, 8, "seed address");
        lam[s * ls + 2 * y] = (float)(2 * ar);
        lam[s * ls + 2 * y + 1] = (float)(2 * ai);
      }
  }
  void pg_rot_bwd(float* psi, float* lam, int nb, int sample0, int r, int slot, const float*, const float*, float* partF) {
    const int q = c.S.runs[r].q;
    const int64_t st = int64_t(1) << q;
    for (int s = 0; s < nb; ++s) {
      float* P = psi + s * 2 * c.amps;
      float* Lm = lam + s * 2 * c.amps;
      double fx = 0, fy = 0, fz = 0;
      for (int64_t i = 0; i < c.amps; ++i) {
        if (i & st) continue;
        const int64_t j = i | st;
        double p0r = P[2 * i], p0i = P[2 * i + 1], p1r = P[2 * j], p1i = P[2 * j + 1];
        double l0r = Lm[2 * i], l0i = Lm[2 * i + 1], l1r = Lm[2 * j], l1i = Lm[2 * j + 1];
        fx += l0r * p1i - l0i * p1r + l1r * p0i - l1i * p0r;
        fy += -(l0r * p1r + l0i * p1i) + (l1r * p0r + l1i * p0i);
        fz += (l0r * p0i - l0i * p0r) - (l1r * p1i - l1i * p1r);
      }
      float* dst = partF + (((int64_t)s * c.pg_chunk + slot) * c.pg_blocks) * 3;
      for (int b = 0; b < c.pg_blocks; ++b) {
        dst[3 * b] = b == 0 ? (float)fx : 0.f;
        dst[3 * b + 1] = b == 0 ? (float)fy : 0.f;
        dst[3 * b + 2] = b == 0 ? (float)fz : 0.f;
      }
      const float* u = coef_row(c.S.runs[r].coef, sample0 + s);
      float ud[8] = {u[0], -u[1], u[4], -u[5], u[2], -u[3], u[6], -u[7]};
      apply1(P, q, ud);
      apply1(Lm, q, ud);
    }
  }
  void pg_assemble(int r0, int cnt, int nb, int sample0, const float*, const float*, const float* partF, float* Gr) {
    for (int s = 0; s < nb; ++s)
      for (int i = 0; i < cnt; ++i) {
        const int r = r0 + i, slot = r % c.pg_chunk;
        double f[3] = {0, 0, 0};
        for (int b = 0; b < c.pg_blocks; ++b)
          for (int P = 0; P < 3; ++P) f[P] += partF[(((int64_t)s * c.pg_chunk + slot) * c.pg_blocks + b) * 3 + P];
        run_grads(r, sample0 + s, f[0], f[1], f[2], Gr + (int64_t)s * c.n_angle, false);
      }
  }
};

thread_local std::string g_err;

}  // namespace
}  // namespace qf

using namespace qf;

extern "C" {

// Runs forward and backward for a circuit on host arrays through the planner's
// programs.  Returns 0 on success, otherwise a qf_status with qfc_last_error().
int qfc_run_psi0(const qf_circuit_desc* desc, int32_t batch, const qf_tuning* tuning, const float* theta,
                 const float* x, const float* psi0, const float* dE, float* E, float* dtheta, float* dx) {
  try {
    std::string msg;
    qf_status st = validate_circuit(desc, &msg);
    if (st != QF_OK) { g_err = msg; return st; }
    Circuit C;
    circuit_from_desc(desc, &C);
    Tuning T;
    if (tuning) {
      T.mode = tuning->mode; T.k = tuning->tile_qubits; T.R = tuning->reg_qubits; T.fusion = tuning->fusion_depth;
      T.ckpt = tuning->ckpt_interval; T.micro = tuning->micro_batch; T.store = tuning->store_ckpt; T.memsave = tuning->mem_save; T.fill = tuning->epoch_fill; T.uncompute = tuning->uncompute;
    }
    if (T.mode == 2) { g_err = "the checker runs float plans only"; return QF_ERR_UNSUPPORTED; }
    PlanCore pc;
    st = build_plan_core(C, batch, T, &pc, &msg);
    if (st != QF_OK) { g_err = msg; return st; }
    std::vector<char> ws(pc.ws_bytes + 256, 0);
    char* base = ws.data();
    CpuExec ex(pc);
    ex.ws_lo = base;
    ex.ws_hi = base + pc.ws_bytes;
    if (psi0) {
      ex.in_lo = (const char*)psi0;
      ex.in_hi = ex.in_lo + pc.state_bytes * batch;
    }
    run_forward(pc, ex, theta, x, E, base, psi0);
    if (dE) run_backward(pc, ex, theta, x, dE, dtheta, dx, base, psi0);
    return 0;
  } catch (const std::exception& e) {
    g_err = e.what();
    return QF_ERR_INTERNAL;
  }
}

int qfc_run(const qf_circuit_desc* desc, int32_t batch, const qf_tuning* tuning, const float* theta,
            const float* x, const float* dE, float* E, float* dtheta, float* dx) {
  return qfc_run_psi0(desc, batch, tuning, theta, x, nullptr, dE, E, dtheta, dx);
}

// Schedule statistics: passes, segments, ops, layout count.
// Worst LDS bank-slot sharing of a plan's tile exchanges: for every PERM (single
// or inside an epoch, forward and backward programs), both its write and its
// read layout, every wave and register slot, the largest number of distinct
// elements that the 32 lanes of one LDS cycle (8-byte accesses: 256 bytes from
// 64 banks) place in one 8-byte bank slot.  1 means conflict-free; lanes that
// read the same element share it.
static int64_t lds_bank_degree(const Schedule& S) {
  const int NA = 1 << S.R, tb = S.thread_bits;
  auto side = [&](const LayoutRec& L) {
    int64_t worst = 1;
    for (int w = 0; w < std::max(1, S.NT / 64); ++w)
      for (int jj = 0; jj < NA; ++jj)
        for (int half = 0; half < 2; ++half) {
          std::vector<std::vector<uint32_t>> slot(32);
          for (int ln = half * 32; ln < half * 32 + 32; ++ln) {
            const int t = (w * 64 + ln) & ((1 << tb) - 1);   // lanes above the tile repeat in-tile ones
            uint32_t v = 0;
            for (int b = 0; b < tb; ++b)
              if ((t >> b) & 1) v ^= L.lds_thr[b];
            const uint32_t e = (v ^ reg_index(L.lds_reg, jj)) / kLdsElemBytes;
            std::vector<uint32_t>& sl = slot[e & 31u];
            if (std::find(sl.begin(), sl.end(), e) == sl.end()) sl.push_back(e);
            worst = std::max<int64_t>(worst, (int64_t)sl.size());
          }
        }
    return worst;
  };
  int64_t worst = 1;
  auto perm = [&](int from, int to) {
    worst = std::max(worst, side(S.layouts[from]));
    worst = std::max(worst, side(S.layouts[to]));
  };
  for (const Op& o : S.ops) {
    if (o.kind == OP_PERM) perm(o.a, o.b);
    if (o.kind == OP_EPOCH)
      for (int e = o.a; e < o.a + o.b; ++e) perm(S.epochs[e].perm_from, S.epochs[e].perm_to);
  }
  return worst;
}

int qfc_stats(const qf_circuit_desc* desc, int32_t batch, const qf_tuning* tuning, int64_t* out, int n_out) {
  std::string msg;
  qf_status st = validate_circuit(desc, &msg);
  if (st != QF_OK) { g_err = msg; return st; }
  Circuit C;
  circuit_from_desc(desc, &C);
  Tuning T;
  if (tuning) {
    T.mode = tuning->mode; T.k = tuning->tile_qubits; T.R = tuning->reg_qubits; T.fusion = tuning->fusion_depth;
    T.ckpt = tuning->ckpt_interval; T.micro = tuning->micro_batch; T.store = tuning->store_ckpt; T.memsave = tuning->mem_save; T.fill = tuning->epoch_fill; T.uncompute = tuning->uncompute;
  }
  PlanCore pc;
  st = build_plan_core(C, batch, T, &pc, &msg);
  if (st != QF_OK) { g_err = msg; return st; }
  int64_t v[17] = {pc.P, pc.n_seg, pc.ckpt, pc.mb, pc.S.n_perm, pc.S.n_u2, pc.S.n_cz, (int64_t)pc.S.layouts.size(),
                   (int64_t)pc.S.runs.size(), pc.S.k, pc.S.R, (int64_t)pc.ws_bytes, pc.S.n_diag_thread,
                   pc.S.n_diag_amp, pc.S.NT, pc.S.thread_bits, pc.per_gate ? 1 : lds_bank_degree(pc.S)};
  for (int i = 0; i < n_out && i < 17; ++i) out[i] = v[i];
  return 0;
}

// Mixed batch on the CPU: builds every circuit's plan, records and merges the
// launch sequences exactly as the device library does, checks every job's
// workspace extents, then replays the merged launches job by job with the
// emulated kernels.  Outputs must equal qfc_run of each circuit alone.
// stats (8): fwd_steps, bwd_steps, fwd_launches, bwd_launches, fwd_jobs,
// bwd_jobs, ws_bytes, max jobs in one launch.
int qfc_batch_run(const qf_circuit_desc* const* descs, const int32_t* samples, int32_t n, const qf_tuning* tuning,
                  const float* const* theta, const float* const* x, const float* const* dE, float* const* E,
                  float* const* dtheta, float* const* dx, int64_t* stats) {
  try {
    std::string msg;
    qf_tuning bt;
    std::memset(&bt, 0, sizeof(bt));
    bt.store_ckpt = -1;
    if (tuning) bt = *tuning;
    std::vector<std::unique_ptr<PlanCore>> pcs;
    std::vector<const PlanCore*> cores;
    std::vector<PlanPtrs> ptrs;
    for (int i = 0; i < n; ++i) {
      qf_status st = validate_circuit(descs[i], &msg);
      if (st != QF_OK) { g_err = msg; return st; }
      Circuit C;
      circuit_from_desc(descs[i], &C);
      const qf_tuning ct = batch_plan_tuning(bt, C.n);
      Tuning T;
      T.mode = ct.mode; T.k = ct.tile_qubits; T.R = ct.reg_qubits; T.fusion = ct.fusion_depth;
      T.ckpt = ct.ckpt_interval; T.micro = ct.micro_batch; T.store = ct.store_ckpt; T.memsave = ct.mem_save;
      T.fill = ct.epoch_fill; T.uncompute = ct.uncompute;
      pcs.emplace_back(new PlanCore);
      st = build_plan_core(C, samples[i], T, pcs.back().get(), &msg);
      if (st != QF_OK) { g_err = msg; return st; }
      const PlanCore& c = *pcs.back();
      if (c.S.general_obs) { g_err = "mixed batches take Z-string observables only"; return QF_ERR_UNSUPPORTED; }
      cores.push_back(&c);
      PlanPtrs pp;   // host copies of the tables: only their addresses enter the jobs
      pp.ops = c.S.ops.data(); pp.layouts = c.S.layouts.data(); pp.czg = c.S.czg.data();
      pp.funcs = c.S.funcs.data(); pp.rygs = c.S.rygs.data(); pp.epochs = c.S.epochs.data(); pp.phas = c.S.phas.data(); pp.passes = c.S.passes.data(); pp.pev = c.S.pev.data(); pp.cza = c.S.cza.data();
      ptrs.push_back(pp);
    }
    std::vector<uint64_t> off;
    const uint64_t ws_bytes = batch_layout(cores, &off);
    std::vector<CircProgram> fwd, bwd;
    record_programs(cores, ptrs, off, &fwd, &bwd);
    std::vector<Region> regions;
    for (int i = 0; i < n; ++i) regions.push_back({off[i], off[i] + cores[i]->ws_bytes});
    if (!check_program(fwd, cores, regions, &msg) || !check_program(bwd, cores, regions, &msg)) {
      g_err = msg;
      return QF_ERR_INTERNAL;
    }
    const std::vector<int> order = batch_order(cores);
    Program pf, pb;
    // the groups run one after the other here (a valid order: they share no launch)
    if (!merge_grouped(fwd, cores, order, &pf, &msg) || !merge_grouped(bwd, cores, order, &pb, &msg)) {
      g_err = msg;
      return QF_ERR_UNSUPPORTED;
    }
    std::vector<char> ws(ws_bytes, 0);
    char* base = ws.data();
    std::vector<std::unique_ptr<CpuExec>> ex;
    for (int i = 0; i < n; ++i) {
      ex.emplace_back(new CpuExec(*cores[i]));
      ex.back()->ws_lo = base + off[i];
      ex.back()->ws_hi = base + off[i] + cores[i]->ws_bytes;
    }
    auto rb = [&](auto p) { return p ? reinterpret_cast<decltype(p)>(base + reinterpret_cast<uintptr_t>(p)) : p; };
    auto replay = [&](const Program& P) {
      for (const MergedLaunch& L : P.launches) {
        for (int q = 0; q < L.n_jobs; ++q) {
          if (L.cls >= 0) {
            const PassJob& j = P.pjobs[L.job0 + q];
            PassLaunch pl = P.plaunch[L.job0 + q];
            pl.src0 = rb(pl.src0);
            pl.src1 = rb(pl.src1);
            pl.dst = rb(pl.dst);
            pl.dst2 = rb(pl.dst2);
            pl.dpsi = rb(pl.dpsi);
            pl.partF = rb(pl.partF);
            pl.partE = rb(pl.partE);
            pl.dE = dE ? dE[j.circ] : nullptr;
            ex[j.circ]->pass(pl);
            continue;
          }
          const SmallJob& j = P.sjobs[L.job0 + q];
          CpuExec& e = *ex[j.circ];
          const int c = j.circ;
          switch (j.kind) {
            case SJ_COEF: e.coef(theta[c], x[c], base + off[c]); break;
            case SJ_EVENT: break;   // the emulated coefficient step also fills the phase events
            case SJ_REDUCE_E: e.reduce_E(j.u.re.nb, j.u.re.sample0, rb(j.u.re.partE), E[c]); break;
            case SJ_ASSEMBLE:
              e.assemble(j.u.as.p0 / cores[c]->ckpt, j.u.as.nb, j.u.as.sample0, theta[c], x[c], rb(j.u.as.partF),
                         rb(j.u.as.Gr));
              break;
            case SJ_REDUCE_G:
              e.reduce_grads(j.u.rg.nb, j.u.rg.sample0, rb(j.u.rg.Gr), dtheta[c], dx ? dx[c] : nullptr,
                             j.u.rg.accumulate != 0);
              break;
            default: throw std::runtime_error("unknown small job");
          }
        }
      }
    };
    replay(pf);
    if (dE) replay(pb);
    if (stats) {
      int64_t mx = 0;
      for (const MergedLaunch& L : pf.launches) mx = std::max<int64_t>(mx, L.n_jobs);
      for (const MergedLaunch& L : pb.launches) mx = std::max<int64_t>(mx, L.n_jobs);
      const int64_t v[8] = {pf.steps, pb.steps, (int64_t)pf.launches.size(), (int64_t)pb.launches.size(), pf.jobs,
                            pb.jobs, (int64_t)ws_bytes, mx};
      for (int i = 0; i < 8; ++i) stats[i] = v[i];
    }
    return 0;
  } catch (const std::exception& e) {
    g_err = e.what();
    return QF_ERR_INTERNAL;
  }
}

const char* qfc_last_error(void) { return g_err.c_str(); }

}  // extern "C"
