"""GPU parity: the HIP path (through the C-ABI) against the complex128 oracle.

Tolerances (single-precision state, double-precision oracle):
  |E_gpu - E_oracle| <= 1e-4 elementwise;
  max_i |g_gpu - g_oracle| / max_i |g_oracle| <= 1e-3 for dL/dtheta and dL/dx
  (a normwise relative error: near-zero gradient entries make an elementwise
  relative error meaningless, so the error is scaled by the largest entry).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle, loss_and_grad_E  # noqa: E402
from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import (CZ, RX, RY, RZ, c1, c2, draw_inputs, hea_gates,  # noqa: E402
                                            z_observables)

pytestmark = pytest.mark.gpu

E_TOL = 1e-4
G_TOL = 1e-3


@pytest.fixture(scope="module")
def orc():
    return Oracle()


def rel(a, b):
    d = float(np.abs(np.asarray(a, np.float64) - b).max()) if np.size(b) else 0.0
    s = float(np.abs(b).max()) if np.size(b) else 0.0
    return d / s if s > 0 else d


def gpu_run(n, gates, theta, x, zmask, dE, **tun):
    dev = torch.device("cuda:0")
    circ = qfuse.Circuit(n, gates, len(theta), x.shape[1], zmask)
    plan = qfuse.Plan(circ, x.shape[0], qfuse.make_tuning(**tun) if tun else None)
    ws = plan.new_workspace(dev)
    th = torch.tensor(theta, device=dev)
    xx = torch.tensor(x, device=dev) if x.shape[1] else None
    E = plan.forward(th, xx, ws)
    dth, dx = plan.backward(th, xx, torch.tensor(dE, dtype=torch.float32, device=dev), ws)
    torch.cuda.synchronize()
    return (E.cpu().numpy(), dth.cpu().numpy(), dx.cpu().numpy() if dx is not None else np.zeros_like(x),
            plan)


def compare(orc, n, gates, theta, x, obs_qubits, seed=0, **tun):
    xm, zm = z_observables(obs_qubits)
    dE = np.random.default_rng(seed).normal(size=(x.shape[0], len(obs_qubits))).astype(np.float32)
    E, dth, dx, plan = gpu_run(n, gates, theta, x, zm, dE, **tun)
    Eo, dtho, dxo = orc.backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL, f"E err {np.abs(E - Eo).max():.3e}"
    assert rel(dth, dtho) <= G_TOL, f"dtheta err {rel(dth, dtho):.3e}"
    if x.shape[1]:
        assert rel(dx, dxo) <= G_TOL, f"dx err {rel(dx, dxo):.3e}"
    return plan


def hea_case(n, L, rots, B, seed=21):
    gates = hea_gates(n, L, rots)
    theta, x, _ = draw_inputs(seed, L * len(rots) * n, B, n)
    return gates, theta, x


def test_c1_full(orc):
    w = c1()
    _, gE = loss_and_grad_E(np.zeros((w.batch, 1)), "sum")
    E, dth, dx, _ = gpu_run(w.n_qubits, w.gates, w.theta, w.x, w.zmask, gE.astype(np.float32))
    Eo, dtho, dxo = orc.backward(w.n_qubits, w.gates, w.theta, w.x, w.xmask, w.zmask, gE)
    assert np.abs(E - Eo).max() <= E_TOL
    assert rel(dth, dtho) <= G_TOL and rel(dx, dxo) <= G_TOL


@pytest.mark.parametrize("n,L,rots,B,tun", [
    (1, 3, ("RX", "RY", "RZ"), 3, {}),
    (5, 3, ("RY", "RZ"), 5, {}),
    (7, 4, ("RX", "RY", "RZ"), 3, {"fusion_depth": 2}),
    (10, 3, ("RY", "RZ"), 4, {}),
    (11, 3, ("RX", "RY", "RZ"), 3, {"fusion_depth": 1, "ckpt_interval": 2}),
    (12, 5, ("RY", "RZ"), 6, {}),
    (13, 3, ("RX", "RY", "RZ"), 2, {}),
])
def test_single_tile(orc, n, L, rots, B, tun):
    gates, theta, x = hea_case(n, L, rots, B)
    compare(orc, n, gates, theta, x, [0, n - 1] if n > 1 else [0], **tun)


@pytest.mark.parametrize("n,L,rots,B,tun", [
    (9, 4, ("RY", "RZ"), 3, {"tile_qubits": 7, "reg_qubits": 2}),
    (10, 5, ("RX", "RY", "RZ"), 3, {"tile_qubits": 8, "reg_qubits": 4, "ckpt_interval": 2, "micro_batch": 2}),
    (12, 4, ("RX", "RY", "RZ"), 5, {"tile_qubits": 11, "fusion_depth": 2, "ckpt_interval": 3, "micro_batch": 2}),
    (14, 3, ("RX", "RY", "RZ"), 3, {}),
    (15, 4, ("RY", "RZ"), 2, {"store_ckpt": 0, "micro_batch": 1}),
    (16, 3, ("RX", "RY", "RZ"), 2, {"fusion_depth": 8}),
    (14, 6, ("RY", "RZ"), 2, {"fusion_depth": 12}),   # epochs with up to 3 register-bit phases
    (7, 3, ("RX", "RY", "RZ"), 2, {"tile_qubits": 3, "reg_qubits": 2, "fusion_depth": 2}),   # tiles of a few qubits
    (8, 3, ("RY", "RZ"), 3, {"tile_qubits": 4, "reg_qubits": 4}),
])
def test_multi_tile(orc, n, L, rots, B, tun):
    gates, theta, x = hea_case(n, L, rots, B)
    compare(orc, n, gates, theta, x, [0, 3, n - 1], **tun)


def test_general_gate_list(orc):
    """Random gates: arbitrary CZ pairs (not a ladder), repeated CZs, shared
    angles, input angles in the middle of the circuit."""
    rng = np.random.default_rng(5)
    n, B = 11, 3
    rows = []
    for q in range(n):
        rows.append((RY, q, -1, -1, q))
    for _ in range(120):
        k = int(rng.integers(0, 4))
        q0 = int(rng.integers(0, n))
        if k == CZ:
            q1 = int((q0 + 1 + rng.integers(0, n - 1)) % n)
            rows.append((CZ, q0, q1, -1, -1))
        elif rng.random() < 0.15:
            rows.append((k, q0, -1, -1, int(rng.integers(0, n))))
        else:
            rows.append((k, q0, -1, int(rng.integers(0, 40)), -1))
    gates = np.asarray(rows, dtype=np.int32)
    theta, x, _ = draw_inputs(9, 40, B, n)
    compare(orc, n, gates, theta, x, [0, 5, 10])
    compare(orc, n, gates, theta, x, [0, 5, 10], tile_qubits=8, reg_qubits=3, fusion_depth=2)


@pytest.mark.parametrize("n,L,rots,B,tun", [
    (13, 3, ("RX", "RY", "RZ"), 2, {}),
    (14, 4, ("RX", "RY", "RZ"), 3, {"ckpt_interval": 2, "micro_batch": 2}),
    (15, 4, ("RY", "RZ"), 2, {"store_ckpt": 0, "micro_batch": 1}),
    (12, 5, ("RX", "RY", "RZ"), 4, {"tile_qubits": 8, "reg_qubits": 3, "fusion_depth": 2}),
    (16, 12, ("RX", "RY", "RZ"), 2, {"ckpt_interval": 1000}),   # one segment: psi rebuilt through every pass
])
def test_uncompute(orc, n, L, rots, B, tun):
    """The adjoint passes rebuild psi (no recompute, nothing stored in a segment)."""
    gates, theta, x = hea_case(n, L, rots, B)
    compare(orc, n, gates, theta, x, [0, 3, n - 1], uncompute=1, **tun)


@pytest.mark.parametrize("fill", [-1, 1, 2, 0])
def test_epoch_fill(orc, fill):
    """Each end-of-pass epoch threshold (a ring: partial epochs at pass ends are common)."""
    gates = hea_gates(14, 5, ("RX", "RY", "RZ"), ring=True)
    theta, x, _ = draw_inputs(31, 5 * 3 * 14, 2, 14)
    compare(orc, 14, gates, theta, x, [0, 7, 13], epoch_fill=fill)


def test_ring_and_z_strings(orc):
    n, L, B = 9, 3, 4
    gates = hea_gates(n, L, ("RX", "RY", "RZ"), ring=True)
    theta, x, _ = draw_inputs(3, L * 3 * n, B, n)
    xm = np.zeros(3, np.uint64)
    zm = np.asarray([0b101, (1 << n) - 1, 0b110000010], np.uint64)
    dE = np.random.default_rng(2).normal(size=(B, 3)).astype(np.float32)
    E, dth, dx, _ = gpu_run(n, gates, theta, x, zm, dE)
    Eo, dtho, dxo = orc.backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL
    assert rel(dth, dtho) <= G_TOL and rel(dx, dxo) <= G_TOL


def test_no_inputs_and_empty_circuit(orc):
    n, B = 6, 2
    gates = np.asarray([(RX, 0, -1, 0, -1), (CZ, 0, 1, -1, -1), (RY, 1, -1, 1, -1)], np.int32)
    theta = np.asarray([0.3, 1.2], np.float32)
    x = np.zeros((B, 0), np.float32)
    compare(orc, n, gates, theta, x, [0, 1])
    # no gates at all: E = <0|Z|0> = 1, no gradients
    E, dth, _, _ = gpu_run(3, np.zeros((0, 5), np.int32), np.zeros(0, np.float32), np.zeros((2, 0), np.float32),
                           [1, 2], np.ones((2, 2), np.float32))
    assert np.allclose(E, 1.0)


@pytest.mark.parametrize("n,L,B", [(6, 3, 3), (11, 3, 2)])
def test_per_gate_baseline(orc, n, L, B):
    gates, theta, x = hea_case(n, L, ("RX", "RY", "RZ"), B)
    compare(orc, n, gates, theta, x, [0, 2], mode=1)


def test_c2_sampled(orc):
    """12-qubit, 100-layer HEA at the full batch of 1024 in the default launch
    configuration; E and dL/dx of sampled samples are checked one by one, and
    dL/dtheta on a 16-sample sub-batch."""
    w = c2()
    dev = torch.device("cuda:0")
    _, gE = loss_and_grad_E(np.zeros((w.batch, w.n_obs)), "mean_sum")
    E, dth, dx, _ = gpu_run(w.n_qubits, w.gates, w.theta, w.x, w.zmask, gE.astype(np.float32))
    idx = [0, 1, 511, 1023]
    Eo, _, dxo = orc.backward(w.n_qubits, w.gates, w.theta, w.x[idx], w.xmask, w.zmask, gE[idx])
    assert np.abs(E[idx] - Eo).max() <= E_TOL
    assert rel(dx[idx], dxo) <= G_TOL
    sub = w.x[:16]
    E2, dth2, dx2, _ = gpu_run(w.n_qubits, w.gates, w.theta, sub, w.zmask, gE[:16].astype(np.float32))
    Eo2, dtho2, _ = orc.backward(w.n_qubits, w.gates, w.theta, sub, w.xmask, w.zmask, gE[:16])
    assert rel(dth2, dtho2) <= G_TOL


def test_deterministic(orc):
    gates, theta, x = hea_case(12, 4, ("RX", "RY", "RZ"), 4)
    zm = [1, 2]
    dE = np.ones((4, 2), np.float32)
    a = gpu_run(12, gates, theta, x, zm, dE, tile_qubits=10)
    b = gpu_run(12, gates, theta, x, zm, dE, tile_qubits=10)
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u, v)
