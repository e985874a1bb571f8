/*
 * qfuse.h -- C-ABI of the fused forward / adjoint-gradient simulator for
 * batched parameterised circuits (MI355X, gfx950).
 *
 * Method: "Fast and memory-efficient classical simulation of quantum machine
 * learning via forward and backward gate fusion".  The library simulates a
 * batch of state vectors, |psi_M(b)> = U_M ... U_1 |0...0>, returns the
 * expectation values E[b][k] = <psi_M(b)| O_k |psi_M(b)> (Sec. 2.1) and, given
 * upstream gradients dE[b][k] = dL/dE_k(b), the adjoint-method gradients with
 * respect to every rotation angle (Sec. 2.2, eq. grad_theta, eq.
 * update_adjoint_state, seeded by lambda_M = 2 sum_k g_k O_k psi_M, eq.
 * bwd_exp_val plus the chain rule).  Runs of gates are fused so that each
 * sample's state crosses HBM once per fused pass in the forward path (Sec. 3.2)
 * and in the backward path, where intermediate states are recomputed in
 * registers by un-applying gates (Sec. 3.3).  Only pass outputs inside the
 * active checkpoint segment and one state per segment are stored (Sec. 3.4).
 *
 * Conventions
 *  - Amplitude index x = sum_i x_i 2^i: qubit 0 is the least significant bit
 *    (Sec. 3.1).
 *  - Rotation u(phi) = cos(phi/2) I - i sin(phi/2) P, P in {X, Y, Z}
 *    (Sec. 3.3, step 2).  CZ(c, t) negates amplitudes with bits c and t set.
 *  - All device buffers are float32 and owned by the caller.  The library owns
 *    only host objects (qf_circuit, qf_plan) and small device descriptor tables
 *    that it allocates in qf_plan_create and frees in qf_plan_destroy.
 *  - Calls are asynchronous on the given HIP stream (a hipStream_t passed as
 *    void*, NULL = default stream).  Inputs are never modified.
 *  - Errors are returned as status codes; nothing crosses the ABI as an
 *    exception.  All validation is done on the host before any launch;
 *    qf_last_error() gives a human-readable message for the calling thread.
 *    Launch failures map to QF_ERR_DEVICE; asynchronous device faults surface
 *    at the caller's next synchronisation.  NaN / Inf inputs propagate.
 *  - Circuits and plans are immutable after creation except for the device
 *    tables a plan owns; one stream per concurrent call on the same plan.
 */
#ifndef QFUSE_H
#define QFUSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QF_OK = 0,
  QF_ERR_INVALID_ARG = 1,  /* bad pointer, index out of range, inconsistent sizes   */
  QF_ERR_UNSUPPORTED = 2,  /* valid request this build does not implement          */
  QF_ERR_WORKSPACE = 3,    /* workspace missing or smaller than qf_workspace_size  */
  QF_ERR_OOM = 4,          /* host or device allocation of plan tables failed      */
  QF_ERR_DEVICE = 5,       /* a HIP call or kernel launch failed                   */
  QF_ERR_INTERNAL = 6
} qf_status;

/* Gate kinds (Sec. 3.1): Pauli rotations, CZ and CNOT (q0 = control, q1 =
   target).  A CNOT is simulated as RY_t(-pi/2), CZ(c, t), RY_t(pi/2) on its
   target t, which the planner fuses with the neighbouring rotations and
   diagonal gates like any other gate (the paper's fused CNOT of App. B.1 moves
   amplitudes instead). */
typedef enum { QF_RX = 0, QF_RY = 1, QF_RZ = 2, QF_CZ = 3, QF_CNOT = 4 } qf_gate_kind;

/*
 * One gate.  Layout-compatible with int32[5].
 *  - rotations: q0 = target qubit, q1 = -1; the angle is theta[theta_idx] when
 *    theta_idx >= 0, else x[b][input_idx] (an input-encoding angle, per sample);
 *    exactly one of the two indices is >= 0.
 *  - CZ, CNOT: q0 != q1, both in [0, n_qubits); theta_idx = input_idx = -1.
 * An angle index used by several gates receives the sum of their gradients.
 */
typedef struct { int32_t kind, q0, q1, theta_idx, input_idx; } qf_gate;

/* Pauli-string observable: X on x_mask bits, Z on z_mask bits (Y on both),
   i.e. i^{#Y} X^{x_mask} Z^{z_mask} (App. B.2).  Z strings (x_mask == 0) are
   evaluated inside the last fused pass.  A circuit with any X or Y factor has its
   trailing diagonal gates applied too (they do not commute with X or Y), and E
   and the adjoint seed are formed from the stored output state by separate
   kernels.  Mixed batches (qf_batch_create) take Z strings only. */
typedef struct { uint64_t x_mask, z_mask; } qf_pauli;

typedef struct {
  int32_t n_qubits;         /* 1..30 (state of 2^n complex64 per sample)         */
  int32_t n_params;         /* length of theta                                    */
  int32_t n_inputs;         /* features per sample (row length of x)              */
  const qf_gate* gates;     /* n_gates gates in application order                 */
  int64_t n_gates;
  const qf_pauli* obs;      /* n_obs observables; E has n_obs columns             */
  int32_t n_obs;
} qf_circuit_desc;

/* Execution modes (qf_tuning.mode). */
typedef enum {
  QF_MODE_FUSED = 0,     /* fused forward and adjoint passes, complex64 (the method)      */
  QF_MODE_PER_GATE = 1,  /* one kernel per gate, complex64: the unfused baseline          */
  QF_MODE_C128 = 2       /* one kernel per gate, complex128, double inputs and outputs:
                            validation only, called through qf_forward_c128 /
                            qf_backward_c128; the other tuning fields except micro_batch
                            are ignored                                                   */
} qf_mode;

/* Execution choices.  0 (or -1 for store_ckpt) selects the built-in default. */
typedef struct {
  int32_t mode;             /* qf_mode: 0 fused, 1 per-gate baseline, 2 complex128     */
  int32_t tile_qubits;      /* k: amplitudes per workgroup tile = 2^k, k <= 13         */
  int32_t reg_qubits;       /* r: register-resident qubits per lane (1..5)             */
  int32_t fusion_depth;     /* max rotation runs applied to one qubit in one pass      */
  int32_t ckpt_interval;    /* fused passes per checkpoint segment                     */
  int32_t micro_batch;      /* samples per backward micro-batch                        */
  int32_t store_ckpt;       /* 1 = forward keeps segment checkpoints for the batch,
                               0 = backward re-runs the forward per micro-batch        */
  int32_t mem_save;         /* memory-saving mode (Sec. 3.2, Sec. 3.4): 1 = the pass
                               outputs stored inside the active checkpoint segment are
                               kept as bfloat16 pairs (4 bytes per amplitude, rounded
                               to nearest even) and widened on load; checkpoints and
                               all arithmetic stay float32.  Expectations are
                               unchanged; gradients carry the rounding of the stored
                               states.  Fused mode only; 0 = off                       */
  int32_t epoch_fill;       /* planner: a register epoch at the end of a fused pass
                               that would hold fewer than epoch_fill runs is left to
                               the next pass (fewer, fuller epochs for more passes).
                               0 = default: reg_qubits (every partial epoch waits)
                               for a plan, -1 for the plans of a mixed batch (whose
                               merged launches favour fewer passes); -1 = none
                               waits, 1..5 = that threshold.  Results are identical
                               up to float rounding order                              */
  int32_t uncompute;        /* backward state reconstruction: 0 = the paper's scheme
                               (each checkpoint segment is recomputed forward and its
                               pass outputs stored, Sec. 3.3-3.4); 1 = every fused
                               adjoint pass also writes psi at its input, un-applied
                               in registers as the pass already does for its gates
                               (reversibility, Sec. 3.3), so the backward recomputes
                               and stores nothing; each segment starts again from its
                               exact checkpoint, so float32 drift spans one segment.
                               Fused mode only, not with mem_save                      */
} qf_tuning;

/* Static description of a plan, for accounting and roofline reporting. */
typedef struct {
  int32_t n_qubits, tile_qubits, reg_qubits, threads, tiles;
  int32_t fused_passes;       /* forward passes for one sample                       */
  int32_t segments;           /* checkpoint segments                                 */
  int32_t ckpt_interval, micro_batch, store_ckpt, fusion_depth;
  int32_t mem_save;           /* stored pass outputs in bfloat16 (qf_tuning.mem_save)  */
  int32_t epoch_fill;         /* threshold the planner used (qf_tuning.epoch_fill)   */
  int32_t uncompute;          /* qf_tuning.uncompute                                 */
  int64_t n_runs;             /* fused single-qubit runs                              */
  int64_t n_perm, n_u2, n_cz; /* ops per sample summed over forward passes            */
  double fwd_bytes_per_sample;   /* algorithmic HBM bytes, forward                    */
  double bwd_bytes_per_sample;   /* algorithmic HBM bytes, backward incl. recompute   */
  double fwd_flops_per_sample;   /* algorithmic flops, forward: 16 per amplitude and
                                    fused run (one 2x2 complex matrix per run)        */
  double bwd_flops_per_sample;   /* algorithmic flops, backward incl. recompute: 48 per
                                    amplitude and run in the adjoint pass             */
  double bwd_pass_bytes_per_sample;  /* bytes of the fused adjoint pass kernel only   */
  double bwd_pass_flops_per_sample;  /* flops of the fused adjoint pass kernel only   */
  int64_t bwd_pass_launches;         /* adjoint pass launches per backward call       */
  double exec_bwd_pass_flops_per_sample;  /* fp32 flops the adjoint pass kernel executes
                                             for the rotations and functionals          */
} qf_plan_info;

typedef struct qf_circuit qf_circuit;
typedef struct qf_plan qf_plan;

/*
 * The parameterised circuit U(theta, x) = U_M ... U_1 of Sec. 2.1 as a gate
 * list, with the observables O_k of the expectation values.  Validates and
 * copies the description (host only; desc and its arrays stay the caller's).
 * Errors: QF_ERR_INVALID_ARG for NULL pointers, qubit or angle indices out of
 * range, a rotation with both or neither angle index, a two-qubit gate on one
 * qubit; QF_ERR_UNSUPPORTED for n_qubits outside 1..30 or more than 64
 * observables.  Ownership of *out passes to the caller; release with
 * qf_circuit_destroy (NULL is accepted).
 */
qf_status qf_circuit_create(const qf_circuit_desc* desc, qf_circuit** out);
qf_status qf_circuit_destroy(qf_circuit* circuit);

/*
 * Builds the execution plan of a circuit for `batch` >= 1 samples: consecutive
 * single-qubit gates on one qubit merged into runs, runs fused into passes that
 * each read and write a sample's state once (forward and backward gate fusion,
 * Sec. 3.2 and Sec. 3.3; fused CZ, App. B.1), and checkpoint segments of
 * passes with the workspace they need (gradient checkpointing, Sec. 3.4, whose
 * memory model is eq. mem_cap_proposed).  Uploads the plan's descriptor tables
 * to the current HIP device, which the later calls must also use.  tuning may
 * be NULL (defaults); it is copied.  Errors: QF_ERR_INVALID_ARG (NULL circuit or
 * out, batch < 1, a tuning field out of range or an invalid combination),
 * QF_ERR_UNSUPPORTED (no kernel for the tile shape, or a pass whose LDS exceeds
 * the device limit: lower fusion_depth), QF_ERR_OOM (host or device allocation
 * of the tables).  Ownership of *out passes to the caller; qf_plan_destroy
 * frees the plan and its device tables (NULL is accepted).
 */
qf_status qf_plan_create(const qf_circuit* circuit, int32_t batch, const qf_tuning* tuning,
                         qf_plan** out);
qf_status qf_plan_destroy(qf_plan* plan);
/* Fills *info (host struct, caller-owned); QF_ERR_INVALID_ARG on NULL. */
qf_status qf_plan_get_info(const qf_plan* plan, qf_plan_info* info);

/*
 * Device workspace in bytes that qf_forward and qf_backward need: segment
 * checkpoints and the stored pass outputs of one segment (Sec. 3.4, eq.
 * mem_cap_proposed with fused passes in place of layers), forward and adjoint
 * working states, partial sums and coefficient tables.  The caller allocates
 * it (start 256-byte aligned) and owns it.  QF_ERR_INVALID_ARG on NULL.
 */
qf_status qf_workspace_size(const qf_plan* plan, size_t* bytes);

/*
 * Forward pass: E[b][k] = <psi_M(b)| O_k |psi_M(b)> with psi_M(b) = U(theta,
 * x_b) |0...0> (Sec. 2.1), the circuit applied in fused passes (Sec. 3.2).
 * theta: device float[n_params]; x: device float[batch][n_inputs], row-major
 * (may be NULL when n_inputs == 0); E: device float[batch][n_obs], row-major,
 * overwritten.  ws: the caller's workspace of ws_bytes >= qf_workspace_size;
 * it must stay untouched until the matching qf_backward has been enqueued.
 * Errors: QF_ERR_INVALID_ARG (NULL plan or buffer, a plan of another device or
 * a complex128 plan), QF_ERR_WORKSPACE (ws NULL, too small or misaligned),
 * QF_ERR_DEVICE (a launch failed).
 */
qf_status qf_forward(qf_plan* plan, const float* theta, const float* x, float* E,
                     void* ws, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): qf_forward with the
 * workspace taken from a library-owned device array of QF_NOALLOC_SCRATCH_BYTES
 * (64 MiB), one per GPU, held from module load until the process ends.  Same
 * arguments, kernels and results as qf_forward (bit for bit); the call allocates
 * nothing and records no profiling events.  Every call on a GPU shares that GPU's
 * array and leaves its contents there, so calls that overlap on one GPU (several
 * streams or host threads) race and must be ordered by the caller; no
 * qf_backward can follow this call (its checkpoints live in the shared array).
 * Errors: those of qf_forward, QF_ERR_WORKSPACE when qf_workspace_size of the
 * plan exceeds QF_NOALLOC_SCRATCH_BYTES (use qf_forward), QF_ERR_DEVICE when the
 * array's device address cannot be obtained.
 */
#define QF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
qf_status qf_forward_noalloc(qf_plan* plan, const float* theta, const float* x, float* E, void* stream);

/*
 * Backward pass by the adjoint method (Sec. 2.2): the adjoint state is seeded as
 * lambda_M = 2 sum_k dE_k O_k psi_M (eq. bwd_exp_val with the chain rule), each
 * angle's gradient is Re<lambda_j| dU_j/dphi |psi_{j-1}> (eq. grad_theta) and
 * lambda is carried back by U_j^dagger (eq. update_adjoint_state), in fused
 * adjoint passes (Sec. 3.3) over checkpoint segments (Sec. 3.4).
 * dE: device float[batch][n_obs] = dL/dE, row-major.  Writes
 *   dtheta: device float[n_params] = sum over the batch (overwritten),
 *   dx:     device float[batch][n_inputs], row-major (overwritten; may be NULL).
 * Needs the same ws, theta and x as the preceding qf_forward on this plan.
 * Errors as qf_forward.
 */
qf_status qf_backward(qf_plan* plan, const float* theta, const float* x, const float* dE,
                      float* dtheta, float* dx, void* ws, size_t ws_bytes, void* stream);

/*
 * The same calls from given initial states instead of |0...0> (the paper's own
 * experiments start from random states, Sec. 4).  psi0: device complex64
 * [batch][2^n_qubits], interleaved (re, im), amplitude index x = sum_i x_i 2^i;
 * not normalised by the library.  The first fused pass reads it in place; the
 * backward reads it again to recompute the first checkpoint segment, so it
 * must be the same buffer, unchanged, in the matching qf_backward_psi0.  No
 * gradient is formed with respect to psi0.  psi0 == NULL is |0...0>, i.e.
 * qf_forward / qf_backward.
 */
qf_status qf_forward_psi0(qf_plan* plan, const float* theta, const float* x, const float* psi0,
                          float* E, void* ws, size_t ws_bytes, void* stream);
qf_status qf_backward_psi0(qf_plan* plan, const float* theta, const float* x, const float* psi0,
                           const float* dE, float* dtheta, float* dx, void* ws, size_t ws_bytes,
                           void* stream);

/*
 * Complex128 validation path (plans created with mode QF_MODE_C128).  The same
 * quantities as qf_forward / qf_backward (Sec. 2.1 expectations; Sec. 2.2
 * adjoint gradients, eq. grad_theta and eq. update_adjoint_state) computed in
 * double precision throughout, one kernel per gate: the state is complex128 and
 * theta, x, E, dE, dtheta and dx are device double arrays with the layouts of
 * the float calls.  Each gate's gradient is taken at the cut after the gate
 * (dL/dtheta = 1/2 Im<lambda|P|psi>) before the gate is un-applied from psi and
 * lambda.  Meant for checking the float paths and for finite-difference
 * gradient checks, not for speed.  The float calls reject such a plan with
 * QF_ERR_INVALID_ARG, and these calls reject any other plan the same way.
 * Workspace: qf_workspace_size of the plan (final states of the batch, two
 * working states per micro-batch sample, partial sums, coefficient tables).
 * psi0: device complex128 [batch][2^n_qubits] initial states, or NULL for
 * |0...0> (the backward needs no psi0: it starts from the stored final states).
 */
qf_status qf_forward_c128(qf_plan* plan, const double* theta, const double* x, const double* psi0,
                          double* E, void* ws, size_t ws_bytes, void* stream);
qf_status qf_backward_c128(qf_plan* plan, const double* theta, const double* x, const double* dE,
                           double* dtheta, double* dx, void* ws, size_t ws_bytes, void* stream);

/*
 * Kernel timing for accounting (the measurements of Sec. 4 as per-kernel time).  While enabled, every launch the plan makes is
 * bracketed by HIP events recorded on the call's stream; qf_profile_read waits
 * for the recorded events, returns per-class launch counts and summed durations
 * (milliseconds) since the last read, and clears them.  Classes: 0 = fused
 * forward pass, 1 = fused adjoint pass, 2 = every other kernel of the plan.
 */
typedef struct {
  int64_t launches[3];
  double ms[3];
} qf_profile;
qf_status qf_profile_enable(qf_plan* plan, int enable);
qf_status qf_profile_read(qf_plan* plan, qf_profile* out);

/*
 * Mixed batches: many different circuits, each with its own parameters, inputs
 * and sample count, simulated together.  Every circuit computes exactly what
 * qf_forward / qf_backward compute for it alone (same sections of the method,
 * same plan, same kernels and the same rounding); only the launches are shared.
 * Each circuit's launch sequence is merged step by step with the others, so one
 * device launch runs the step's pass of every circuit at that step, and the
 * whole merged sequence can be replayed as one HIP graph.
 *
 * Ownership: the batch owns one plan per circuit, the merged launch tables on
 * the device and a small pinned host buffer; the circuits may be destroyed after
 * qf_batch_create.  The caller owns every buffer passed to the calls.
 */
typedef struct qf_batch qf_batch;

typedef enum {
  QF_LAUNCH_GRAPH = 0,        /* merged launches, captured once per workspace address
                                 into a HIP graph and replayed (default)              */
  QF_LAUNCH_MERGED = 1,       /* the same merged launches, issued one by one          */
  QF_LAUNCH_PER_CIRCUIT = 2   /* each circuit's own launches, circuit after circuit
                                 (the unmerged reference point)                       */
} qf_launch_mode;

typedef struct {
  int32_t n_circuits;
  int64_t samples;             /* sum over circuits                                   */
  int32_t fwd_steps, bwd_steps;          /* longest launch sequence of one circuit    */
  int64_t fwd_launches, bwd_launches;    /* merged launches per call                  */
  int64_t fwd_jobs, bwd_jobs;            /* launches when circuits run one by one     */
  double fwd_bytes, bwd_bytes;           /* algorithmic HBM bytes of one call, summed */
  double fwd_flops, bwd_flops;           /* algorithmic fp32 flops of one call, summed */
} qf_batch_info;

/*
 * circuits[i] is simulated for samples[i] >= 1 samples; each gets the plan that
 * qf_plan_create would build (Sec. 3.2-3.4: runs fused into passes,
 * checkpoint segments), and the plans' launch sequences are merged: circuits
 * of one tile shape share launches, and the shapes run on concurrent streams.
 * tuning (may be NULL) applies to every circuit's plan, with batch defaults for
 * its zero fields (epoch_fill -1, i.e. no end-of-pass epoch waits; fusion_depth
 * 12 for circuits larger than one tile), since every pass costs a merged step;
 * mode must be 0 (fused); mem_save may be set.  Errors: QF_ERR_INVALID_ARG (NULL or empty arrays,
 * samples < 1), QF_ERR_UNSUPPORTED (mode != 0, X or Y factors in an
 * observable, or any qf_plan_create refusal, named by circuit index),
 * QF_ERR_OOM.  The plans and merged tables live on the current HIP device.
 */
qf_status qf_batch_create(const qf_circuit* const* circuits, const int32_t* samples, int32_t n_circuits,
                          const qf_tuning* tuning, qf_batch** out);
qf_status qf_batch_destroy(qf_batch* batch);
qf_status qf_batch_get_info(const qf_batch* batch, qf_batch_info* info);
/* One device workspace for the whole batch (256-byte aligned start expected). */
qf_status qf_batch_workspace_size(const qf_batch* batch, size_t* bytes);
qf_status qf_batch_set_launch_mode(qf_batch* batch, int32_t mode);

/*
 * Forward of every circuit: qf_forward's expectations (Sec. 2.1) per circuit.
 * theta, x and E are HOST arrays of n_circuits
 * DEVICE pointers: theta[i] float[n_params_i], x[i] float[samples_i][n_inputs_i]
 * (NULL allowed when n_inputs_i == 0), E[i] float[samples_i][n_obs_i],
 * overwritten.  The batch copies the pointer arrays before returning.
 * Calls on one batch must be ordered (one stream, or synchronised streams).
 */
qf_status qf_batch_forward(qf_batch* batch, const float* const* theta, const float* const* x,
                           float* const* E, void* ws, size_t ws_bytes, void* stream);

/*
 * Backward of every circuit: qf_backward's adjoint gradients (Sec. 2.2, eq.
 * grad_theta, eq. update_adjoint_state) per circuit, after qf_batch_forward
 * with the same ws, theta and x.  dE[i] float[samples_i][n_obs_i]; dtheta[i] float[n_params_i] (overwritten,
 * summed over the circuit's samples); dx may be NULL, or dx[i] NULL, or
 * dx[i] float[samples_i][n_inputs_i] (overwritten).
 */
qf_status qf_batch_backward(qf_batch* batch, const float* const* theta, const float* const* x,
                            const float* const* dE, float* const* dtheta, float* const* dx, void* ws,
                            size_t ws_bytes, void* stream);

const char* qf_status_string(qf_status status);
/* Detail of the last error on the calling thread ("" if none). */
const char* qf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QFUSE_H */
