"""CNOT gates (control q0, target q1) through the CPU execution of the planner's
programs, against the oracle's textbook CNOT: HEA ladders and rings of CNOT,
mixed CZ / CNOT lists with rotations on both ends, fused and per gate."""
import numpy as np
import pytest

import plancheck as pc
from oracle.oracle import Oracle
from paper_2603_02804_amd.workloads import CNOT, CZ, RX, RY, RZ, draw_inputs, hea_gates, z_observables
from pauli_cases import strings

E_TOL, G_TOL = 1e-4, 1e-3


def rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("n,L,ring,mode,tun", [
    (14, 3, False, 0, {}),
    (13, 4, True, 0, dict(ckpt_interval=2)),
    (9, 3, True, 0, {}),
    (8, 3, False, 1, {}),
])
def test_cnot_hea(n, L, ring, mode, tun):
    gates = hea_gates(n, L, ("RX", "RY", "RZ"), ring=ring, entangler=CNOT)
    theta, x, _ = draw_inputs(120 + n, L * 3 * n, 2, n)
    xm, zm = strings(n)
    dE = np.random.default_rng(n).normal(size=(2, len(zm)))
    E, dth, dx = pc.run(n, gates, theta, x, zm, dE, xmask=xm, mode=mode, **tun)
    Eo, dtho, dxo = Oracle().backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL
    assert rel(dth, dtho) <= G_TOL and rel(dx, dxo) <= G_TOL


def test_cnot_random_lists():
    rng = np.random.default_rng(9)
    n, B = 11, 2
    rows = [(RY, q, -1, -1, q) for q in range(n)]
    for _ in range(150):
        k = int(rng.integers(0, 5))
        q0 = int(rng.integers(0, n))
        if k in (CZ, CNOT):
            rows.append((k, q0, int((q0 + 1 + rng.integers(0, n - 1)) % n), -1, -1))
        else:
            rows.append((k, q0, -1, int(rng.integers(0, 30)), -1))
    gates = np.asarray(rows, dtype=np.int32)
    theta, x, _ = draw_inputs(11, 30, B, n)
    xm, zm = z_observables([0, 5, 10])
    dE = rng.normal(size=(B, 3))
    E, dth, dx = pc.run(n, gates, theta, x, zm, dE)
    Eo, dtho, dxo = Oracle().backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL
    assert rel(dth, dtho) <= G_TOL and rel(dx, dxo) <= G_TOL
