"""General Pauli-string observables (X, Y and Z factors, App. B.2) through the
CPU execution of the planner's programs, fused and per gate, against the
oracle: the last fused pass applies the trailing diagonal gates (they do not
commute with X or Y), and E and the adjoint seed come from the stored output
state in its own bit order."""
import numpy as np
import pytest

import plancheck as pc
from oracle.oracle import Oracle
from paper_2603_02804_amd.workloads import draw_inputs, hea_gates
from pauli_cases import strings

E_TOL, G_TOL = 1e-4, 1e-3


def rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("n,L,mode,tun", [
    (14, 3, 0, {}),
    (14, 3, 0, dict(ckpt_interval=1, micro_batch=1)),
    (13, 5, 0, dict(mem_save=1, ckpt_interval=2)),
    (13, 5, 0, dict(uncompute=1, ckpt_interval=2)),
    (9, 4, 0, {}),
    (10, 2, 1, {}),
])
def test_pauli_observables(n, L, mode, tun):
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    theta, x, _ = draw_inputs(70 + n, L * 3 * n, 2, n)
    xm, zm = strings(n)
    dE = np.random.default_rng(n).normal(size=(2, len(zm)))
    E, dth, dx = pc.run(n, gates, theta, x, zm, dE, xmask=xm, mode=mode, **tun)
    Eo, dtho, dxo = Oracle().backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL
    assert rel(dth, dtho) <= G_TOL and rel(dx, dxo) <= G_TOL


def test_z_strings_keep_the_fused_expectation():
    # Z-only observables take the path with E fused into the last pass and no
    # trailing diagonal gates applied: the same numbers either way
    n, L = 14, 3
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    theta, x, _ = draw_inputs(3, L * 3 * n, 2, n)
    zm = np.array([1, 1 << 13, 0b1010], np.uint64)
    dE = np.random.default_rng(0).normal(size=(2, 3))
    E, dth, dx = pc.run(n, gates, theta, x, zm, dE)
    Eo, dtho, dxo = Oracle().backward(n, gates, theta, x, np.zeros(3, np.uint64), zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL and rel(dth, dtho) <= G_TOL
