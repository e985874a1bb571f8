"""The C-ABI library on the CPU: it loads, exports every entry point the header
declares, and rejects invalid requests on the host before touching a device.

No call here launches a kernel: circuit creation is host-only, and every plan
or call below fails host-side validation before any HIP call is made.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2603_02804_amd import qfuse

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]

QF_OK, INVALID, UNSUPPORTED, WORKSPACE = 0, 1, 2, 3


def declared_functions():
    names = set()
    for path in HEADERS:
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(qf_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return qfuse.library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("qf_circuit_create", "qf_plan_create", "qf_forward", "qf_backward", "qf_forward_c128",
              "qf_backward_c128", "qf_batch_create", "qf_batch_forward", "qf_batch_backward"):
        assert n in names


def test_library_exports_every_declared_function(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_status_strings(lib):
    for code, text in qfuse._STATUS.items():
        assert qfuse.qf_status_string(code) == text
    assert qfuse.qf_status_string(99) == "unknown status"


def _desc(n, gates, P=1, F=0, z=(1,), x=None):
    g = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 5)
    obs = np.zeros((len(z), 2), dtype=np.uint64)
    obs[:, 1] = z
    if x is not None:
        obs[:, 0] = x
    d = qfuse.qf_circuit_desc(n, P, F, g.ctypes.data, len(g), obs.ctypes.data if len(z) else None, len(z))
    return d, (g, obs)


def _create(lib, desc):
    h = ctypes.c_void_p()
    st = lib.qf_circuit_create(ctypes.byref(desc) if desc is not None else None, ctypes.byref(h))
    return st, h


RX, RY, RZ, CZ = 0, 1, 2, 3


@pytest.mark.parametrize("n,gates,P,F,z,x,want", [
    (2, [[RY, 0, -1, 0, -1]], 1, 0, (1,), None, QF_OK),
    (0, [[RY, 0, -1, 0, -1]], 1, 0, (1,), None, UNSUPPORTED),           # no qubits
    (31, [[RY, 0, -1, 0, -1]], 1, 0, (1,), None, UNSUPPORTED),          # beyond 30 qubits
    (2, [[7, 0, -1, 0, -1]], 1, 0, (1,), None, INVALID),                # unknown kind
    (2, [[RY, 2, -1, 0, -1]], 1, 0, (1,), None, INVALID),               # qubit out of range
    (2, [[CZ, 0, 0, -1, -1]], 1, 0, (1,), None, INVALID),               # CZ on one qubit
    (2, [[CZ, 0, 2, -1, -1]], 1, 0, (1,), None, INVALID),               # CZ partner out of range
    (2, [[CZ, 0, 1, 0, -1]], 1, 0, (1,), None, INVALID),                # CZ with an angle
    (2, [[4, 1, 0, -1, -1]], 1, 0, (1,), None, QF_OK),                  # CNOT 1 -> 0
    (2, [[4, 1, 1, -1, -1]], 1, 0, (1,), None, INVALID),                # CNOT on one qubit
    (2, [[4, 0, 1, 0, -1]], 1, 0, (1,), None, INVALID),                 # CNOT with an angle
    (2, [[5, 0, 1, -1, -1]], 1, 0, (1,), None, INVALID),                # unknown two-qubit kind
    (2, [[RY, 0, -1, 0, 0]], 1, 1, (1,), None, INVALID),                # two angle sources
    (2, [[RY, 0, -1, -1, -1]], 1, 0, (1,), None, INVALID),              # no angle source
    (2, [[RY, 0, -1, 1, -1]], 1, 0, (1,), None, INVALID),               # theta_idx >= n_params
    (2, [[RY, 0, -1, -1, 3]], 1, 3, (1,), None, INVALID),               # input_idx >= n_inputs
    (2, [[RY, 0, -1, 0, -1]], 1, 0, (4,), None, INVALID),               # observable beyond the register
    (2, [[RY, 0, -1, 0, -1]], 1, 0, (1,), (1,), QF_OK),                 # Y on qubit 0
    (2, [[RY, 0, -1, 0, -1]], 1, 0, (0,), (3,), QF_OK),                 # XX
    (2, [[RY, 0, -1, 0, -1]], 1, 0, (0,), (4,), INVALID),               # X beyond the register
])
def test_circuit_validation(lib, n, gates, P, F, z, x, want):
    desc, _keep = _desc(n, gates, P, F, z, x)
    st, h = _create(lib, desc)
    assert st == want, lib.qf_last_error()
    if st == QF_OK:
        assert lib.qf_circuit_destroy(h) == QF_OK
    else:
        assert h.value is None
        assert len(lib.qf_last_error()) > 0


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.qf_circuit_create(None, ctypes.byref(h)) == INVALID
    assert lib.qf_plan_create(None, 1, None, ctypes.byref(h)) == INVALID
    assert lib.qf_forward(None, None, None, None, None, 0, None) == INVALID
    assert lib.qf_forward_noalloc(None, None, None, None, None) == INVALID
    assert lib.qf_backward(None, None, None, None, None, None, None, 0, None) == INVALID
    assert lib.qf_forward_psi0(None, None, None, None, None, None, 0, None) == INVALID
    assert lib.qf_backward_psi0(None, None, None, None, None, None, None, None, 0, None) == INVALID
    assert lib.qf_forward_c128(None, None, None, None, None, None, 0, None) == INVALID
    assert lib.qf_backward_c128(None, None, None, None, None, None, None, 0, None) == INVALID
    assert lib.qf_workspace_size(None, None) == INVALID
    assert lib.qf_plan_get_info(None, None) == INVALID
    assert lib.qf_plan_destroy(None) == QF_OK
    assert lib.qf_circuit_destroy(None) == QF_OK


@pytest.mark.parametrize("batch,tuning", [
    (0, None),                                            # empty batch
    (1, qfuse.make_tuning(mode=3)),                       # unknown mode
    (1, qfuse.make_tuning(tile_qubits=14)),               # tile beyond 2^13 amplitudes
    (1, qfuse.make_tuning(reg_qubits=6)),                 # more register qubits than supported
    (1, qfuse.make_tuning(ckpt_interval=-1)),             # negative value
    (1, qfuse.make_tuning(mem_save=2)),                   # mem_save is a flag
    (1, qfuse.make_tuning(mode=1, mem_save=1)),           # memory-saving mode is for fused plans
    (1, qfuse.make_tuning(epoch_fill=-2)),                # epoch threshold below -1
    (1, qfuse.make_tuning(epoch_fill=6)),                 # epoch threshold beyond the register
    (1, qfuse.make_tuning(uncompute=2)),                  # uncompute is a flag
    (1, qfuse.make_tuning(mode=1, uncompute=1)),          # uncompute is for fused plans
    (1, qfuse.make_tuning(uncompute=1, mem_save=1)),      # nothing stored to compress
])
def test_plan_validation_before_any_device_call(lib, batch, tuning):
    desc, _keep = _desc(2, [[RY, 0, -1, 0, -1], [CZ, 0, 1, -1, -1]])
    st, circ = _create(lib, desc)
    assert st == QF_OK
    try:
        h = ctypes.c_void_p()
        st = lib.qf_plan_create(circ, batch, ctypes.byref(tuning) if tuning is not None else None, ctypes.byref(h))
        assert st == INVALID
        assert h.value is None
    finally:
        lib.qf_circuit_destroy(circ)


def test_plan_refused_when_a_pass_exceeds_the_lds_limit(lib):
    """A fusion depth that puts thousands of runs into one pass would need more LDS
    per adjoint-pass workgroup (per-wave functional sums) than any device has: the
    plan is refused at creation (host-side check, before any upload or launch)."""
    from paper_2603_02804_amd.workloads import hea_gates
    n, L = 12, 2000
    gates = hea_gates(n, L, ("RY",), encoding=False)
    desc, _keep = _desc(n, gates, P=n * L)
    st, circ = _create(lib, desc)
    assert st == QF_OK
    try:
        h = ctypes.c_void_p()
        t = qfuse.make_tuning(tile_qubits=12, reg_qubits=4, fusion_depth=L)
        st = lib.qf_plan_create(circ, 1, ctypes.byref(t), ctypes.byref(h))
        assert st == UNSUPPORTED, lib.qf_last_error()
        assert h.value is None
        assert b"LDS" in lib.qf_last_error()
    finally:
        lib.qf_circuit_destroy(circ)
