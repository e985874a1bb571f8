"""Python binding of the C-ABI in include/qfuse.h (argument marshalling only).

The functions ``qf_*`` below carry the C names and take the same arguments, with
device buffers given as torch tensors (their data pointers are passed through).
``Plan`` and ``CircuitFunction`` are conveniences built from them; every step of
the simulation runs in the HIP library.  Importing this module does not load the
library; the first call does, and fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

from .build import LIB

QF_OK = 0
# qf_tuning.mode
QF_MODE_FUSED, QF_MODE_PER_GATE, QF_MODE_C128 = 0, 1, 2
_STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "workspace too small", 4: "out of memory",
           5: "device error", 6: "internal error"}


class QFuseError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{_STATUS.get(status, status)}: {detail}")
        self.status = status


class qf_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("theta_idx", ctypes.c_int32), ("input_idx", ctypes.c_int32)]


class qf_pauli(ctypes.Structure):
    _fields_ = [("x_mask", ctypes.c_uint64), ("z_mask", ctypes.c_uint64)]


class qf_circuit_desc(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_params", ctypes.c_int32), ("n_inputs", ctypes.c_int32),
                ("gates", ctypes.c_void_p), ("n_gates", ctypes.c_int64), ("obs", ctypes.c_void_p),
                ("n_obs", ctypes.c_int32)]


class qf_tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("mode", "tile_qubits", "reg_qubits", "fusion_depth",
                                              "ckpt_interval", "micro_batch", "store_ckpt", "mem_save",
                                              "epoch_fill", "uncompute")]


class qf_plan_info(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int32) for n in ("n_qubits", "tile_qubits", "reg_qubits", "threads", "tiles",
                                               "fused_passes", "segments", "ckpt_interval", "micro_batch",
                                               "store_ckpt", "fusion_depth", "mem_save", "epoch_fill",
                                               "uncompute")]
                + [("n_runs", ctypes.c_int64), ("n_perm", ctypes.c_int64), ("n_u2", ctypes.c_int64),
                   ("n_cz", ctypes.c_int64)]
                + [(n, ctypes.c_double) for n in ("fwd_bytes_per_sample", "bwd_bytes_per_sample",
                                                  "fwd_flops_per_sample", "bwd_flops_per_sample",
                                                  "bwd_pass_bytes_per_sample", "bwd_pass_flops_per_sample")]
                + [("bwd_pass_launches", ctypes.c_int64), ("exec_bwd_pass_flops_per_sample", ctypes.c_double)])


class qf_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 3), ("ms", ctypes.c_double * 3)]


QF_LAUNCH_GRAPH, QF_LAUNCH_MERGED, QF_LAUNCH_PER_CIRCUIT = 0, 1, 2


class qf_batch_info(ctypes.Structure):
    _fields_ = [("n_circuits", ctypes.c_int32), ("samples", ctypes.c_int64),
                ("fwd_steps", ctypes.c_int32), ("bwd_steps", ctypes.c_int32),
                ("fwd_launches", ctypes.c_int64), ("bwd_launches", ctypes.c_int64),
                ("fwd_jobs", ctypes.c_int64), ("bwd_jobs", ctypes.c_int64),
                ("fwd_bytes", ctypes.c_double), ("bwd_bytes", ctypes.c_double),
                ("fwd_flops", ctypes.c_double), ("bwd_flops", ctypes.c_double)]


_lib = None


def library() -> ctypes.CDLL:
    """The HIP library; raises if it is missing (there is no other execution path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise FileNotFoundError(f"{LIB} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB)
        P, I32, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        sigs = {
            "qf_circuit_create": [P, P], "qf_circuit_destroy": [P],
            "qf_plan_create": [P, I32, P, P], "qf_plan_destroy": [P], "qf_plan_get_info": [P, P],
            "qf_workspace_size": [P, P],
            "qf_forward": [P, P, P, P, P, SZ, P],
            "qf_forward_noalloc": [P, P, P, P, P],
            "qf_backward": [P, P, P, P, P, P, P, SZ, P],
            "qf_forward_psi0": [P, P, P, P, P, P, SZ, P],
            "qf_backward_psi0": [P, P, P, P, P, P, P, P, SZ, P],
            "qf_forward_c128": [P, P, P, P, P, P, SZ, P],
            "qf_backward_c128": [P, P, P, P, P, P, P, SZ, P],
            "qf_profile_enable": [P, ctypes.c_int], "qf_profile_read": [P, P],
            "qf_batch_create": [P, P, I32, P, P], "qf_batch_destroy": [P], "qf_batch_get_info": [P, P],
            "qf_batch_workspace_size": [P, P], "qf_batch_set_launch_mode": [P, I32],
            "qf_batch_forward": [P, P, P, P, P, SZ, P],
            "qf_batch_backward": [P, P, P, P, P, P, P, SZ, P],
        }
        for name, args in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.qf_status_string.restype = ctypes.c_char_p
        lib.qf_status_string.argtypes = [ctypes.c_int]
        lib.qf_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def _check(status: int) -> None:
    if status != QF_OK:
        raise QFuseError(status, library().qf_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# --------------------------------------------------------------------- C names
def qf_circuit_create(desc: qf_circuit_desc) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(library().qf_circuit_create(ctypes.byref(desc), ctypes.byref(h)))
    return h


def qf_circuit_destroy(circuit) -> None:
    _check(library().qf_circuit_destroy(circuit))


def qf_plan_create(circuit, batch: int, tuning: Optional[qf_tuning]) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(library().qf_plan_create(circuit, int(batch), ctypes.byref(tuning) if tuning else None, ctypes.byref(h)))
    return h


def qf_plan_destroy(plan) -> None:
    _check(library().qf_plan_destroy(plan))


def qf_plan_get_info(plan) -> qf_plan_info:
    info = qf_plan_info()
    _check(library().qf_plan_get_info(plan, ctypes.byref(info)))
    return info


def qf_workspace_size(plan) -> int:
    n = ctypes.c_size_t()
    _check(library().qf_workspace_size(plan, ctypes.byref(n)))
    return int(n.value)


def qf_forward(plan, theta: torch.Tensor, x: Optional[torch.Tensor], E: torch.Tensor, ws: torch.Tensor,
               ws_bytes: int, stream) -> None:
    _check(library().qf_forward(plan, _ptr(theta), _ptr(x), _ptr(E), _ptr(ws), ws_bytes, stream))


def qf_forward_noalloc(plan, theta: torch.Tensor, x: Optional[torch.Tensor], E: torch.Tensor, stream) -> None:
    _check(library().qf_forward_noalloc(plan, _ptr(theta), _ptr(x), _ptr(E), stream))


def qf_backward(plan, theta: torch.Tensor, x: Optional[torch.Tensor], dE: torch.Tensor, dtheta: torch.Tensor,
                dx: Optional[torch.Tensor], ws: torch.Tensor, ws_bytes: int, stream) -> None:
    _check(library().qf_backward(plan, _ptr(theta), _ptr(x), _ptr(dE), _ptr(dtheta), _ptr(dx), _ptr(ws),
                                 ws_bytes, stream))


def qf_forward_psi0(plan, theta: torch.Tensor, x: Optional[torch.Tensor], psi0: Optional[torch.Tensor],
                    E: torch.Tensor, ws: torch.Tensor, ws_bytes: int, stream) -> None:
    _check(library().qf_forward_psi0(plan, _ptr(theta), _ptr(x), _ptr(psi0), _ptr(E), _ptr(ws), ws_bytes, stream))


def qf_backward_psi0(plan, theta: torch.Tensor, x: Optional[torch.Tensor], psi0: Optional[torch.Tensor],
                     dE: torch.Tensor, dtheta: torch.Tensor, dx: Optional[torch.Tensor], ws: torch.Tensor,
                     ws_bytes: int, stream) -> None:
    _check(library().qf_backward_psi0(plan, _ptr(theta), _ptr(x), _ptr(psi0), _ptr(dE), _ptr(dtheta), _ptr(dx),
                                      _ptr(ws), ws_bytes, stream))


def qf_forward_c128(plan, theta: torch.Tensor, x: Optional[torch.Tensor], psi0: Optional[torch.Tensor],
                    E: torch.Tensor, ws: torch.Tensor, ws_bytes: int, stream) -> None:
    _check(library().qf_forward_c128(plan, _ptr(theta), _ptr(x), _ptr(psi0), _ptr(E), _ptr(ws), ws_bytes, stream))


def qf_backward_c128(plan, theta: torch.Tensor, x: Optional[torch.Tensor], dE: torch.Tensor, dtheta: torch.Tensor,
                     dx: Optional[torch.Tensor], ws: torch.Tensor, ws_bytes: int, stream) -> None:
    _check(library().qf_backward_c128(plan, _ptr(theta), _ptr(x), _ptr(dE), _ptr(dtheta), _ptr(dx), _ptr(ws),
                                      ws_bytes, stream))


def qf_profile_enable(plan, enable: bool) -> None:
    _check(library().qf_profile_enable(plan, 1 if enable else 0))


def qf_profile_read(plan) -> qf_profile:
    out = qf_profile()
    _check(library().qf_profile_read(plan, ctypes.byref(out)))
    return out


def qf_status_string(status: int) -> str:
    return library().qf_status_string(status).decode()


# --------------------------------------------------------------------- conveniences
def make_tuning(mode=0, tile_qubits=0, reg_qubits=0, fusion_depth=0, ckpt_interval=0, micro_batch=0,
                store_ckpt=-1, mem_save=0, epoch_fill=0, uncompute=0) -> qf_tuning:
    return qf_tuning(mode, tile_qubits, reg_qubits, fusion_depth, ckpt_interval, micro_batch, store_ckpt, mem_save,
                     epoch_fill, uncompute)


class Circuit:
    """Owns a qf_circuit built from int32 gate rows (kind, q0, q1, theta_idx, input_idx)."""

    def __init__(self, n_qubits: int, gates, n_params: int, n_inputs: int, z_masks: Sequence[int],
                 x_masks: Optional[Sequence[int]] = None):
        self.gates = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 5)
        K = len(z_masks)
        self.obs = np.zeros((K, 2), dtype=np.uint64)
        self.obs[:, 1] = np.asarray(z_masks, dtype=np.uint64)
        if x_masks is not None:
            self.obs[:, 0] = np.asarray(x_masks, dtype=np.uint64)
        self.n_qubits, self.n_params, self.n_inputs, self.n_obs = n_qubits, n_params, n_inputs, K
        desc = qf_circuit_desc(n_qubits, n_params, n_inputs, self.gates.ctypes.data, len(self.gates),
                               self.obs.ctypes.data if K else None, K)
        self.handle = qf_circuit_create(desc)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.qf_circuit_destroy(h)
            self.handle = None


class Plan:
    """A qf_plan for one batch size and tuning, plus its workspace."""

    def __init__(self, circuit: Circuit, batch: int, tuning: Optional[qf_tuning] = None):
        self.circuit = circuit
        self.batch = int(batch)
        # tuning mode 2: the complex128 validation path (float64 inputs and outputs)
        self.c128 = tuning is not None and tuning.mode == QF_MODE_C128
        self.dtype = torch.float64 if self.c128 else torch.float32
        self.handle = qf_plan_create(circuit.handle, self.batch, tuning)
        self.ws_bytes = qf_workspace_size(self.handle)

    @property
    def info(self) -> qf_plan_info:
        return qf_plan_get_info(self.handle)

    def new_workspace(self, device=None) -> torch.Tensor:
        return torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device or "cuda")

    def _check_inputs(self, theta, x):
        c, dt = self.circuit, self.dtype
        if theta.dtype != dt or not theta.is_cuda or theta.numel() != c.n_params:
            raise ValueError(f"theta must be a {dt} CUDA tensor of n_params elements")
        if c.n_inputs:
            if x is None or x.dtype != dt or not x.is_cuda or tuple(x.shape) != (self.batch, c.n_inputs):
                raise ValueError(f"x must be a {dt} CUDA tensor of shape [batch, n_inputs]")

    def _check_psi0(self, psi0):
        if psi0 is None:
            return None
        want = torch.complex128 if self.c128 else torch.complex64
        if psi0.dtype != want or not psi0.is_cuda or tuple(psi0.shape) != (self.batch, 1 << self.circuit.n_qubits):
            raise ValueError(f"psi0 must be a {want} CUDA tensor of shape [batch, 2^n_qubits]")
        return torch.view_as_real(psi0.contiguous())

    def forward(self, theta: torch.Tensor, x: Optional[torch.Tensor], ws: torch.Tensor,
                E: Optional[torch.Tensor] = None, psi0: Optional[torch.Tensor] = None) -> torch.Tensor:
        """psi0: initial states (complex, [batch, 2^n]); None is |0...0>."""
        self._check_inputs(theta, x)
        p0 = self._check_psi0(psi0)
        theta = theta.contiguous()
        x = x.contiguous() if x is not None else None
        if E is None:
            E = torch.empty(self.batch, self.circuit.n_obs, dtype=self.dtype, device=theta.device)
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        if self.c128:
            qf_forward_c128(self.handle, theta, x, p0, E, ws, ws.numel(), s)
        else:
            qf_forward_psi0(self.handle, theta, x, p0, E, ws, ws.numel(), s)
        return E

    def forward_noalloc(self, theta: torch.Tensor, x: Optional[torch.Tensor],
                        E: Optional[torch.Tensor] = None) -> torch.Tensor:
        """qf_forward_noalloc: the forward with the library's own device array as workspace
        (no backward can follow; calls on one GPU must not overlap)."""
        self._check_inputs(theta, x)
        if self.c128:
            raise ValueError("qf_forward_noalloc takes float32 plans only")
        theta = theta.contiguous()
        x = x.contiguous() if x is not None else None
        if E is None:
            E = torch.empty(self.batch, self.circuit.n_obs, dtype=self.dtype, device=theta.device)
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        qf_forward_noalloc(self.handle, theta, x, E, s)
        return E

    def backward(self, theta: torch.Tensor, x: Optional[torch.Tensor], dE: torch.Tensor, ws: torch.Tensor,
                 want_dx: bool = True, psi0: Optional[torch.Tensor] = None):
        """psi0: the same initial states as the forward (None: |0...0>)."""
        self._check_inputs(theta, x)
        p0 = self._check_psi0(psi0)
        dE = dE.contiguous().to(self.dtype)
        # the library writes dense row-major outputs: allocate them so, whatever the inputs' strides
        dtheta = torch.empty(theta.shape, dtype=self.dtype, device=theta.device)
        dx = torch.empty(x.shape, dtype=self.dtype, device=x.device) if (want_dx and x is not None) else None
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        xc = x.contiguous() if x is not None else None
        if self.c128:
            qf_backward_c128(self.handle, theta.contiguous(), xc, dE, dtheta, dx, ws, ws.numel(), s)
        else:
            qf_backward_psi0(self.handle, theta.contiguous(), xc, p0, dE, dtheta, dx, ws, ws.numel(), s)
        return dtheta, dx

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.qf_plan_destroy(h)
            self.handle = None


class CircuitFunction(torch.autograd.Function):
    """E = circuit(theta, x) with the fused adjoint backward.

    The forward keeps the plan's workspace (segment checkpoints) alive in the
    autograd context; the backward re-runs each segment from its checkpoint and
    returns dL/dtheta (summed over the batch) and dL/dx (per sample).  Inputs are
    never modified.  The workspace is released after the first backward unless
    ``retain_workspace`` is set (needed when the graph is differentiated more
    than once, as torch.autograd.gradcheck does).
    """

    @staticmethod
    def forward(ctx, theta, x, plan: Plan, retain_workspace: bool = False, psi0=None):
        ws = plan.new_workspace(theta.device)
        E = plan.forward(theta.detach(), x.detach() if x is not None else None, ws, psi0=psi0)
        ctx.plan = plan
        ctx.ws = ws
        # psi0 is saved like the other inputs: the backward reads it again (the first
        # segment's recompute), so an in-place change in between must raise
        empty = torch.empty(0, device=theta.device)
        ctx.save_for_backward(theta, x if x is not None else empty, psi0 if psi0 is not None else empty)
        ctx.has_x = x is not None
        ctx.has_psi0 = psi0 is not None
        ctx.retain = bool(retain_workspace)
        return E

    @staticmethod
    def backward(ctx, gE):
        theta, x, psi0 = ctx.saved_tensors
        x = x if ctx.has_x else None
        psi0 = psi0 if ctx.has_psi0 else None
        want_dx = ctx.has_x and ctx.needs_input_grad[1]
        dtheta, dx = ctx.plan.backward(theta.detach(), x.detach() if x is not None else None, gE, ctx.ws,
                                       want_dx=want_dx, psi0=psi0)
        if not ctx.retain:
            ctx.ws = None
        return dtheta, dx, None, None, None


def circuit_expectations(theta: torch.Tensor, x: Optional[torch.Tensor], plan: Plan,
                         retain_workspace: bool = False, psi0: Optional[torch.Tensor] = None) -> torch.Tensor:
    """E = circuit(theta, x) from |0...0> or from the initial states psi0 (no gradient w.r.t. psi0)."""
    return CircuitFunction.apply(theta, x, plan, retain_workspace, psi0)


# --------------------------------------------------------------------- mixed batches
def _ptr_array(ts) -> ctypes.Array:
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def qf_batch_create(circuits, samples, tuning: Optional[qf_tuning]) -> ctypes.c_void_p:
    n = len(circuits)
    hs = (ctypes.c_void_p * n)(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in circuits])
    ss = (ctypes.c_int32 * n)(*[int(v) for v in samples])
    h = ctypes.c_void_p()
    _check(library().qf_batch_create(hs, ss, n, ctypes.byref(tuning) if tuning else None, ctypes.byref(h)))
    return h


def qf_batch_destroy(batch) -> None:
    _check(library().qf_batch_destroy(batch))


def qf_batch_get_info(batch) -> qf_batch_info:
    info = qf_batch_info()
    _check(library().qf_batch_get_info(batch, ctypes.byref(info)))
    return info


def qf_batch_workspace_size(batch) -> int:
    n = ctypes.c_size_t()
    _check(library().qf_batch_workspace_size(batch, ctypes.byref(n)))
    return int(n.value)


def qf_batch_set_launch_mode(batch, mode: int) -> None:
    _check(library().qf_batch_set_launch_mode(batch, int(mode)))


def qf_batch_forward(batch, thetas, xs, Es, ws: torch.Tensor, ws_bytes: int, stream) -> None:
    _check(library().qf_batch_forward(batch, _ptr_array(thetas), _ptr_array(xs), _ptr_array(Es), _ptr(ws),
                                      int(ws_bytes), stream))


def qf_batch_backward(batch, thetas, xs, dEs, dthetas, dxs, ws: torch.Tensor, ws_bytes: int, stream) -> None:
    _check(library().qf_batch_backward(batch, _ptr_array(thetas), _ptr_array(xs), _ptr_array(dEs),
                                       _ptr_array(dthetas), _ptr_array(dxs) if dxs is not None else None, _ptr(ws),
                                       int(ws_bytes), stream))


class Batch:
    """A qf_batch over several circuits with their own sample counts."""

    def __init__(self, circuits: Sequence[Circuit], samples: Sequence[int], tuning: Optional[qf_tuning] = None,
                 launch_mode: int = QF_LAUNCH_GRAPH):
        self.circuits = list(circuits)
        self.samples = [int(s) for s in samples]
        if len(self.samples) != len(self.circuits):
            raise ValueError("one sample count per circuit")
        self.handle = qf_batch_create([c.handle for c in self.circuits], self.samples, tuning)
        self.ws_bytes = qf_batch_workspace_size(self.handle)
        self.set_launch_mode(launch_mode)

    def set_launch_mode(self, mode: int) -> None:
        qf_batch_set_launch_mode(self.handle, mode)

    @property
    def info(self) -> qf_batch_info:
        return qf_batch_get_info(self.handle)

    def new_workspace(self, device=None) -> torch.Tensor:
        return torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device or "cuda")

    def _check(self, thetas, xs):
        if len(thetas) != len(self.circuits) or len(xs) != len(self.circuits):
            raise ValueError("one theta and one x per circuit")
        for c, s, t, x in zip(self.circuits, self.samples, thetas, xs):
            if t.dtype != torch.float32 or not t.is_cuda or t.numel() != c.n_params or not t.is_contiguous():
                raise ValueError("theta: contiguous float32 CUDA tensor of n_params elements per circuit")
            if c.n_inputs and (x is None or x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous()
                               or tuple(x.shape) != (s, c.n_inputs)):
                raise ValueError("x: contiguous float32 CUDA tensor [samples, n_inputs] per circuit")

    def forward(self, thetas, xs, ws: torch.Tensor):
        self._check(thetas, xs)
        Es = [torch.empty(s, c.n_obs, dtype=torch.float32, device=ws.device)
              for c, s in zip(self.circuits, self.samples)]
        qf_batch_forward(self.handle, thetas, xs, Es, ws, ws.numel(),
                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        return Es

    def backward(self, thetas, xs, dEs, ws: torch.Tensor, want_dx: bool = True):
        self._check(thetas, xs)
        dEs = [d.contiguous().to(torch.float32) for d in dEs]
        dthetas = [torch.empty_like(t) for t in thetas]
        dxs = [torch.empty_like(x) if (want_dx and x is not None) else None for x in xs]
        qf_batch_backward(self.handle, thetas, xs, dEs, dthetas, dxs, ws, ws.numel(),
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        return dthetas, dxs

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.qf_batch_destroy(h)
            self.handle = None
