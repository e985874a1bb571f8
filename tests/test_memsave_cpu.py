"""Memory-saving mode through the CPU execution of the planner's programs: the
expectations are those of the float32 path bit for bit, the gradients stay
within the rounding bound of bfloat16 storage (tests/memsave_bound.py) around
the oracle, and the workspace shrinks by half of the stored pass outputs."""
import numpy as np
import pytest

import plancheck as pc
from memsave_bound import gradient_bounds, lambda_norms
from oracle.oracle import Oracle
from paper_2603_02804_amd.workloads import draw_inputs, hea_gates, z_observables

G_TOL = 1e-3


@pytest.mark.parametrize("n,L,B,ckpt,mb", [(14, 10, 3, 3, 2), (13, 12, 2, 4, 2)])
def test_mem_save_against_oracle(n, L, B, ckpt, mb):
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    P = L * 3 * n
    theta, x, _ = draw_inputs(40 + n, P, B, n)
    xm, zm = z_observables([0, n - 1])
    dE = np.random.default_rng(n).normal(size=(B, 2))
    E0, dth0, dx0 = pc.run(n, gates, theta, x, zm, dE, ckpt_interval=ckpt, micro_batch=mb)
    E1, dth1, dx1 = pc.run(n, gates, theta, x, zm, dE, ckpt_interval=ckpt, micro_batch=mb, mem_save=1)
    assert np.array_equal(E0, E1)
    assert not np.array_equal(dth0, dth1)          # the rounding is really there
    orc = Oracle()
    _, dtho, dxo = orc.backward(n, gates, theta, x, xm, zm, dE)
    lam = lambda_norms(orc, n, gates, theta, x, zm, dE)
    bth, bx = gradient_bounds(gates, P, n, lam)
    allow_th = G_TOL * np.abs(dtho).max()
    allow_x = G_TOL * np.abs(dxo).max()
    assert np.all(np.abs(dth1 - dtho) <= bth + allow_th)
    assert np.all(np.abs(dx1 - dxo) <= bx + allow_x)


def test_mem_save_workspace():
    n, L, B = 14, 12, 8
    g = hea_gates(n, L, ("RX", "RY", "RZ"))
    full = pc.stats(n, g, L * 3 * n, n, [1], B, ckpt_interval=5, micro_batch=4)
    half = pc.stats(n, g, L * 3 * n, n, [1], B, ckpt_interval=5, micro_batch=4, mem_save=1)
    stored = (full["ckpt"] - 1) * full["micro_batch"] * (8 << n)
    assert full["ws_bytes"] - half["ws_bytes"] == pytest.approx(stored / 2, abs=4096)
