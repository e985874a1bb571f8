/*
 * qfo.c -- CPU oracle for batched state-vector simulation with adjoint gradients.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference against which the GPU
 * path is checked.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the GPU library, and it never calls into it.
 *
 * What it computes (paper: "Fast and memory-efficient classical simulation of
 * quantum machine learning via forward and backward gate fusion"):
 *
 *  - State vector of n qubits, complex128, amplitude index x = sum_i x_i 2^i,
 *    qubit 0 is the least significant bit (Sec. 3.1).
 *  - A single-qubit gate u on target t updates every pair of amplitudes whose
 *    indices differ only in bit t: (a0, a1) <- u (a0, a1)  (Sec. 3.1).
 *  - CZ(c, t) negates the amplitudes whose bits c and t are both 1 (Sec. 3.1).
 *  - CNOT(c, t) flips bit t of every basis state whose bit c is 1: it swaps the
 *    amplitudes x and x ^ 2^t for every x with bit c set (Sec. 3.1, the fused
 *    CNOT of App. B.1 is this permutation of the state's indices).
 *  - Pauli rotations u(phi) = cos(phi/2) I - i sin(phi/2) P, with derivative
 *    du/dphi = -1/2 sin(phi/2) I - i/2 cos(phi/2) P  (Sec. 3.3, step 2).
 *  - Expectation E = <psi_M| O |psi_M> (Sec. 2.1) for Pauli strings O given by
 *    an X mask and a Z mask (a Y sits where both bits are set); the action
 *    (O psi)_x = i^{nY} (-1)^{popcount((x ^ xm) & zm)} psi_{x ^ xm} follows
 *    App. B.2 (computing expectation values).
 *  - Adjoint method (Sec. 2.2): lambda_M = 2 O psi_M for L = E (eq.
 *    bwd_exp_val); with several observables and an upstream gradient
 *    g_k = dL/dE_k the chain rule gives lambda_M = 2 sum_k g_k O_k psi_M.
 *    Then for j = M..1:  dL/dtheta_j = Re <lambda_j| dU_j/dtheta_j |psi_{j-1}>
 *    (eq. grad_theta) and lambda_{j-1} = U_j^dagger lambda_j
 *    (eq. update_adjoint_state).
 *
 * Two backward modes, cross-checked by the tests:
 *   mode 0: recover psi_{j-1} = U_j^dagger psi_j by un-applying gates;
 *   mode 1: store every psi_j during the forward sweep (small cases only).
 *
 * Gate encoding (this file's own): int32 quintuples
 *   { kind, q0, q1, theta_idx, input_idx }, kind 0=RX 1=RY 2=RZ 3=CZ 4=CNOT
 *   (q0 = control, q1 = target).
 * A rotation takes its angle from theta[theta_idx] if theta_idx >= 0, else from
 * x[b][input_idx].  Gradients of an angle used by several gates are summed;
 * dtheta is summed over the batch, dx is per sample.
 *
 * All arithmetic is in double.  Callers pass float32 inputs promoted exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { QFO_RX = 0, QFO_RY = 1, QFO_RZ = 2, QFO_CZ = 3, QFO_CNOT = 4 };

typedef struct { double re, im; } cplx;

static cplx c_make(double re, double im) { cplx z; z.re = re; z.im = im; return z; }
static cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static cplx c_mul(cplx a, cplx b) { return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static cplx c_conj(cplx a) { return c_make(a.re, -a.im); }
static cplx c_scale(cplx a, double s) { return c_make(a.re * s, a.im * s); }

/* 2x2 complex matrix, row-major: m[0]=u00 m[1]=u01 m[2]=u10 m[3]=u11 */
typedef struct { cplx m[4]; } mat2;

/* The Pauli matrix P for a rotation kind. */
static mat2 pauli(int kind) {
  mat2 p;
  int i;
  for (i = 0; i < 4; ++i) p.m[i] = c_make(0.0, 0.0);
  if (kind == QFO_RX) {            /* X = [[0,1],[1,0]] */
    p.m[1] = c_make(1.0, 0.0);
    p.m[2] = c_make(1.0, 0.0);
  } else if (kind == QFO_RY) {     /* Y = [[0,-i],[i,0]] */
    p.m[1] = c_make(0.0, -1.0);
    p.m[2] = c_make(0.0, 1.0);
  } else {                         /* Z = [[1,0],[0,-1]] */
    p.m[0] = c_make(1.0, 0.0);
    p.m[3] = c_make(-1.0, 0.0);
  }
  return p;
}

/* u(phi) = cos(phi/2) I - i sin(phi/2) P */
static mat2 rot(int kind, double phi) {
  mat2 p = pauli(kind), u;
  double c = cos(0.5 * phi), s = sin(0.5 * phi);
  int i;
  for (i = 0; i < 4; ++i) {
    /* -i s P */
    u.m[i] = c_mul(c_make(0.0, -s), p.m[i]);
  }
  u.m[0] = c_add(u.m[0], c_make(c, 0.0));
  u.m[3] = c_add(u.m[3], c_make(c, 0.0));
  return u;
}

/* du/dphi = -1/2 sin(phi/2) I - i/2 cos(phi/2) P */
static mat2 drot(int kind, double phi) {
  mat2 p = pauli(kind), d;
  double c = cos(0.5 * phi), s = sin(0.5 * phi);
  int i;
  for (i = 0; i < 4; ++i) d.m[i] = c_mul(c_make(0.0, -0.5 * c), p.m[i]);
  d.m[0] = c_add(d.m[0], c_make(-0.5 * s, 0.0));
  d.m[3] = c_add(d.m[3], c_make(-0.5 * s, 0.0));
  return d;
}

static mat2 dagger(mat2 u) {
  mat2 d;
  d.m[0] = c_conj(u.m[0]);
  d.m[1] = c_conj(u.m[2]);
  d.m[2] = c_conj(u.m[1]);
  d.m[3] = c_conj(u.m[3]);
  return d;
}

/* Apply u to every amplitude pair differing only in bit t. */
static void apply_1q(cplx* psi, int n, int t, mat2 u) {
  int64_t dim = (int64_t)1 << n, step = (int64_t)1 << t, i;
#pragma omp parallel for schedule(static) if (n >= 16)
  for (i = 0; i < dim; ++i) {
    if (i & step) continue;
    cplx a0 = psi[i], a1 = psi[i | step];
    psi[i] = c_add(c_mul(u.m[0], a0), c_mul(u.m[1], a1));
    psi[i | step] = c_add(c_mul(u.m[2], a0), c_mul(u.m[3], a1));
  }
}

/* CZ: negate amplitudes with bits c and t both set. */
static void apply_cz(cplx* psi, int n, int c, int t) {
  int64_t dim = (int64_t)1 << n, i;
  int64_t mc = (int64_t)1 << c, mt = (int64_t)1 << t;
#pragma omp parallel for schedule(static) if (n >= 16)
  for (i = 0; i < dim; ++i)
    if ((i & mc) && (i & mt)) psi[i] = c_scale(psi[i], -1.0);
}

/* CNOT: swap the amplitudes of x and x ^ 2^t wherever bit c of x is 1. */
static void apply_cnot(cplx* psi, int n, int c, int t) {
  int64_t dim = (int64_t)1 << n, i;
  int64_t mc = (int64_t)1 << c, mt = (int64_t)1 << t;
#pragma omp parallel for schedule(static) if (n >= 16)
  for (i = 0; i < dim; ++i)
    if ((i & mc) && !(i & mt)) {
      cplx a = psi[i];
      psi[i] = psi[i | mt];
      psi[i | mt] = a;
    }
}

/* Re <lam| (d applied on bit t) |psi> */
static double grad_term(const cplx* lam, const cplx* psi, int n, int t, mat2 d) {
  int64_t dim = (int64_t)1 << n, step = (int64_t)1 << t, i;
  double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc) if (n >= 16)
  for (i = 0; i < dim; ++i) {
    if (i & step) continue;
    cplx a0 = psi[i], a1 = psi[i | step];
    cplx k0 = c_add(c_mul(d.m[0], a0), c_mul(d.m[1], a1));
    cplx k1 = c_add(c_mul(d.m[2], a0), c_mul(d.m[3], a1));
    acc += c_mul(c_conj(lam[i]), k0).re + c_mul(c_conj(lam[i | step]), k1).re;
  }
  return acc;
}

static int popcount64(uint64_t v) {
  int c = 0;
  while (v) { v &= v - 1; ++c; }
  return c;
}

/* out = O psi for the Pauli string (xm, zm); Y where both bits are set. */
static void apply_pauli_string(const cplx* psi, cplx* out, int n, uint64_t xm, uint64_t zm) {
  int64_t dim = (int64_t)1 << n, i;
  int ny = popcount64(xm & zm) & 3;
  cplx iy = c_make(1.0, 0.0);
  int k;
  for (k = 0; k < ny; ++k) iy = c_mul(iy, c_make(0.0, 1.0));
#pragma omp parallel for schedule(static) if (n >= 16)
  for (i = 0; i < dim; ++i) {
    uint64_t src = (uint64_t)i ^ xm;
    double sgn = (popcount64(src & zm) & 1) ? -1.0 : 1.0;
    out[i] = c_scale(c_mul(iy, psi[src]), sgn);
  }
}

static double angle_of(const int32_t* g, const double* theta, const double* xb) {
  return g[3] >= 0 ? theta[g[3]] : xb[g[4]];
}

static int validate(int n, int n_gates, const int32_t* gates, int n_params, int n_inputs) {
  int j;
  if (n < 1 || n > 30 || n_gates < 0) return 1;
  for (j = 0; j < n_gates; ++j) {
    const int32_t* g = gates + 5 * j;
    if (g[0] < 0 || g[0] > 4) return 2;
    if (g[1] < 0 || g[1] >= n) return 3;
    if (g[0] == QFO_CZ || g[0] == QFO_CNOT) {
      if (g[2] < 0 || g[2] >= n || g[2] == g[1]) return 4;
    } else {
      if ((g[3] >= 0) == (g[4] >= 0)) return 5;
      if (g[3] >= n_params || g[4] >= n_inputs) return 6;
    }
  }
  return 0;
}

/* Run all gates forward on psi (length 2^n) for one sample. */
static void forward_one(cplx* psi, int n, int n_gates, const int32_t* gates,
                        const double* theta, const double* xb, cplx** store) {
  int j;
  if (store) memcpy(store[0], psi, sizeof(cplx) << n);
  for (j = 0; j < n_gates; ++j) {
    const int32_t* g = gates + 5 * j;
    if (g[0] == QFO_CZ) apply_cz(psi, n, g[1], g[2]);
    else if (g[0] == QFO_CNOT) apply_cnot(psi, n, g[1], g[2]);
    else apply_1q(psi, n, g[1], rot(g[0], angle_of(g, theta, xb)));
    if (store) memcpy(store[j + 1], psi, sizeof(cplx) << n);
  }
}

static void init_state(cplx* psi, int n, const double* psi0_b) {
  int64_t dim = (int64_t)1 << n, i;
  if (psi0_b) {
    for (i = 0; i < dim; ++i) psi[i] = c_make(psi0_b[2 * i], psi0_b[2 * i + 1]);
  } else {
    for (i = 0; i < dim; ++i) psi[i] = c_make(0.0, 0.0);
    psi[0] = c_make(1.0, 0.0);
  }
}

static double expect_one(const cplx* psi, cplx* tmp, int n, uint64_t xm, uint64_t zm) {
  int64_t dim = (int64_t)1 << n, i;
  double acc = 0.0;
  apply_pauli_string(psi, tmp, n, xm, zm);
  for (i = 0; i < dim; ++i) acc += c_mul(c_conj(psi[i]), tmp[i]).re;
  return acc;
}

/* Parallelise across samples when there are enough of them and the states are
   small; otherwise run samples one after another and parallelise inside. */
static int across_samples(int n, int B) {
#ifdef _OPENMP
  return n < 16 && B > 1;
#else
  (void)n; (void)B;
  return 0;
#endif
}

/*
 * Forward: E[b][k] = <psi_M(b)| O_k |psi_M(b)>.
 * psi0: optional initial states [B][2^n][2] (NULL = |0...0>).
 * psi_out: optional final states [B][2^n][2].
 * Returns 0 on success, >0 on invalid input, <0 on allocation failure.
 */
int qfo_forward(int n, int n_gates, const int32_t* gates, int n_params, const double* theta,
                int n_inputs, const double* x, int B, const double* psi0,
                int n_obs, const uint64_t* xmask, const uint64_t* zmask,
                double* E, double* psi_out) {
  int b, err = validate(n, n_gates, gates, n_params, n_inputs), fail = 0;
  int64_t dim = (int64_t)1 << n;
  if (err) return err;
  if (B < 0 || n_obs < 0) return 7;
#pragma omp parallel for schedule(dynamic) if (across_samples(n, B)) reduction(| : fail)
  for (b = 0; b < B; ++b) {
    cplx* psi = (cplx*)malloc(sizeof(cplx) * dim);
    cplx* tmp = (cplx*)malloc(sizeof(cplx) * dim);
    int k;
    int64_t i;
    if (!psi || !tmp) { free(psi); free(tmp); fail = 1; continue; }
    init_state(psi, n, psi0 ? psi0 + 2 * dim * b : NULL);
    forward_one(psi, n, n_gates, gates, theta, n_inputs ? x + (int64_t)n_inputs * b : NULL, NULL);
    for (k = 0; k < n_obs; ++k) E[(int64_t)b * n_obs + k] = expect_one(psi, tmp, n, xmask[k], zmask[k]);
    if (psi_out)
      for (i = 0; i < dim; ++i) {
        psi_out[2 * (dim * b + i)] = psi[i].re;
        psi_out[2 * (dim * b + i) + 1] = psi[i].im;
      }
    free(psi);
    free(tmp);
  }
  return fail ? -1 : 0;
}

/*
 * Backward: given upstream gradients dE[b][k] = dL/dE_k(b), return
 *   dtheta[p] = sum_b dL/dtheta_p (overwritten),
 *   dx[b][f]  = dL/dx_{b,f} (overwritten; may be NULL).
 * Also returns E (may be NULL).  mode 0 = un-apply, mode 1 = store-all.
 */
int qfo_backward(int n, int n_gates, const int32_t* gates, int n_params, const double* theta,
                 int n_inputs, const double* x, int B, const double* psi0,
                 int n_obs, const uint64_t* xmask, const uint64_t* zmask,
                 const double* dE, double* dtheta, double* dx, double* E, int mode) {
  int b, p, err = validate(n, n_gates, gates, n_params, n_inputs), fail = 0;
  int64_t dim = (int64_t)1 << n;
  double* gth;
  if (err) return err;
  if (B < 0 || n_obs < 0 || (mode != 0 && mode != 1)) return 7;
  /* per-sample theta gradients, summed over the batch in a fixed order */
  gth = (double*)calloc((size_t)(B > 0 ? B : 1) * (n_params > 0 ? n_params : 1), sizeof(double));
  if (!gth) return -1;
  if (dx) memset(dx, 0, sizeof(double) * (size_t)B * n_inputs);
#pragma omp parallel for schedule(dynamic) if (across_samples(n, B)) reduction(| : fail)
  for (b = 0; b < B; ++b) {
    const double* xb = n_inputs ? x + (int64_t)n_inputs * b : NULL;
    cplx* psi = (cplx*)malloc(sizeof(cplx) * dim);
    cplx* lam = (cplx*)calloc(dim, sizeof(cplx));
    cplx* tmp = (cplx*)malloc(sizeof(cplx) * dim);
    cplx** store = NULL;
    int j, k;
    int64_t i;
    if (!psi || !lam || !tmp) { free(psi); free(lam); free(tmp); fail = 1; continue; }
    if (mode == 1) {
      store = (cplx**)calloc(n_gates + 1, sizeof(cplx*));
      for (j = 0; store && j <= n_gates; ++j) {
        store[j] = (cplx*)malloc(sizeof(cplx) * dim);
        if (!store[j]) { fail = 1; break; }
      }
      if (!store || fail) {
        for (j = 0; store && j <= n_gates; ++j) free(store[j]);
        free(store); free(psi); free(lam); free(tmp);
        fail = 1;
        continue;
      }
    }
    init_state(psi, n, psi0 ? psi0 + 2 * dim * b : NULL);
    forward_one(psi, n, n_gates, gates, theta, xb, store);
    /* lambda_M = 2 sum_k g_k O_k psi_M */
    for (k = 0; k < n_obs; ++k) {
      double g = dE[(int64_t)b * n_obs + k];
      if (E) E[(int64_t)b * n_obs + k] = expect_one(psi, tmp, n, xmask[k], zmask[k]);
      apply_pauli_string(psi, tmp, n, xmask[k], zmask[k]);
      for (i = 0; i < dim; ++i) lam[i] = c_add(lam[i], c_scale(tmp[i], 2.0 * g));
    }
    /* reverse sweep */
    for (j = n_gates - 1; j >= 0; --j) {
      const int32_t* g = gates + 5 * j;
      if (g[0] == QFO_CZ) {
        /* CZ is real and self-adjoint; it has no parameter */
        if (mode == 0) apply_cz(psi, n, g[1], g[2]);
        apply_cz(lam, n, g[1], g[2]);
      } else if (g[0] == QFO_CNOT) {
        /* a permutation that is its own inverse; no parameter */
        if (mode == 0) apply_cnot(psi, n, g[1], g[2]);
        apply_cnot(lam, n, g[1], g[2]);
      } else {
        double phi = angle_of(g, theta, xb);
        mat2 u = rot(g[0], phi);
        const cplx* prev;
        double gr;
        if (mode == 0) {
          apply_1q(psi, n, g[1], dagger(u));    /* psi <- psi_{j-1} */
          prev = psi;
        } else {
          prev = store[j];                       /* psi_{j-1} */
        }
        gr = grad_term(lam, prev, n, g[1], drot(g[0], phi));
        if (g[3] >= 0) gth[(int64_t)b * n_params + g[3]] += gr;
        else if (dx) dx[(int64_t)b * n_inputs + g[4]] += gr;
        apply_1q(lam, n, g[1], dagger(u));       /* lambda <- lambda_{j-1} */
      }
    }
    if (store) {
      for (j = 0; j <= n_gates; ++j) free(store[j]);
      free(store);
    }
    free(psi);
    free(lam);
    free(tmp);
  }
  if (!fail)
    for (p = 0; p < n_params; ++p) {
      double acc = 0.0;
      for (b = 0; b < B; ++b) acc += gth[(int64_t)b * n_params + p];
      dtheta[p] = acc;
    }
  free(gth);
  return fail ? -1 : 0;
}

/* Number of threads the oracle's parallel regions use. */
int qfo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void qfo_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
