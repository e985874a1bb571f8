"""Seeded random circuits and execution choices shared by the CPU and GPU randomised tests
(inputs only: no arithmetic of the method)."""
import numpy as np

from paper_2603_02804_amd.workloads import CNOT, CZ, draw_inputs, hea_gates


def random_circuit(rng, seed, max_n=9):
    """1..max_n qubits, 1..4 layers of a random subset of RX/RY/RZ, CZ or CNOT ladder or
    ring, 1..4 samples, Z observables on qubit 0, the last qubit and a random one."""
    n = int(rng.integers(1, max_n + 1))
    L = int(rng.integers(1, 5))
    rots = tuple(r for r in ("RX", "RY", "RZ") if rng.random() < 0.7) or ("RY",)
    ring = bool(rng.random() < 0.3) and n > 2
    ent = CNOT if rng.random() < 0.3 else CZ
    gates = hea_gates(n, L, rots, ring=ring, entangler=ent)
    B = int(rng.integers(1, 5))
    theta, x, _ = draw_inputs(seed, L * len(rots) * n, B, n)
    obs = sorted({0, n - 1, int(rng.integers(0, n))})
    return n, gates, theta, x, obs


def random_tuning(rng, n, batch):
    k = int(rng.integers(0, n + 1))
    R = int(rng.integers(0, min(max(k, 1), 5) + 1))
    return dict(tile_qubits=k, reg_qubits=R, fusion_depth=int(rng.integers(0, 7)),
                epoch_fill=int(rng.choice([-1, 0, 1, 2, 3])), uncompute=int(rng.integers(0, 2)),
                ckpt_interval=int(rng.integers(0, 4)), micro_batch=int(rng.integers(0, batch + 1)))


def random_tuning_wide(rng, n, batch):
    """Execution choices for 10..16 qubits that the pass kernels support (at most 256
    threads per tile): default, 10..13 tile qubits with 4 or 5 register qubits."""
    k = int(rng.choice([0, 10, 11, 12, 13]))
    R = int(rng.choice([0, 4, 5])) if k != 13 else 5
    return dict(tile_qubits=min(k, n), reg_qubits=R, fusion_depth=int(rng.integers(0, 13)),
                epoch_fill=int(rng.choice([-1, 0, 2, 4])), uncompute=int(rng.integers(0, 2)),
                ckpt_interval=int(rng.integers(0, 4)), micro_batch=int(rng.integers(0, batch + 1)))


def random_batch_tuning(rng):
    return dict(fusion_depth=int(rng.integers(0, 7)), epoch_fill=int(rng.choice([-1, 0, 2])),
                uncompute=int(rng.integers(0, 2)), tile_qubits=int(rng.choice([0, 0, 5, 6, 8])))


def close(E, dth, dx, ref, e_tol=1e-4, g_tol=1e-3):
    """E within e_tol; gradients within g_tol of max(max |ref|, 1e-3), so that gradients that
    vanish analytically (RZ-only layers under Z observables) compare absolutely."""
    Eo, dtho, dxo = ref
    s = max(float(np.abs(dtho).max()), 1e-3) if np.size(dtho) else 1.0
    sx = max(float(np.abs(dxo).max()), 1e-3) if np.size(dxo) else 1.0
    ok = float(np.abs(E - Eo).max()) <= e_tol
    if np.size(dtho):
        ok = ok and float(np.abs(dth - dtho).max()) / s <= g_tol
    if np.size(dxo):
        ok = ok and float(np.abs(dx - dxo).max()) / sx <= g_tol
    return ok
