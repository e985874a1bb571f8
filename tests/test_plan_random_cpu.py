"""Randomised plans on the CPU: seeded random circuits (1-9 qubits, RX/RY/RZ subsets, CZ or
CNOT ladders or rings) under random execution choices (tile and register qubits, fusion
depth, end-of-pass epoch threshold, uncompute mode, checkpoint interval, micro-batch), and
random mixed batches of such circuits, run through the CPU execution of the planner's
programs and compared with the oracle (paper Sec. 2.1 expectation, Sec. 2.2 adjoint
gradient).  Gradients are compared against max(max |dtheta|, 1e-3), so that circuits whose
gradient vanishes analytically (RZ-only layers under Z observables) compare absolutely."""
import numpy as np
import pytest

import plancheck as pc
from oracle.oracle import Oracle
from paper_2603_02804_amd.workloads import CNOT, CZ, draw_inputs, hea_gates, z_observables

E_TOL, G_TOL = 1e-4, 1e-3


@pytest.fixture(scope="module")
def orc():
    return Oracle()


def random_circuit(rng, seed, max_n=9):
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


def close(E, dth, dx, ref):
    Eo, dtho, dxo = ref
    s = max(float(np.abs(dtho).max()), 1e-3)
    sx = max(float(np.abs(dxo).max()), 1e-3)
    return (float(np.abs(E - Eo).max()) <= E_TOL and float(np.abs(dth - dtho).max()) / s <= G_TOL
            and float(np.abs(dx - dxo).max()) / sx <= G_TOL)


@pytest.mark.parametrize("seed", range(200))
def test_random_plan(orc, seed):
    rng = np.random.default_rng(1000 + seed)
    n, gates, theta, x, obs = random_circuit(rng, seed)
    k = int(rng.integers(0, n + 1))
    R = int(rng.integers(0, min(max(k, 1), 5) + 1))
    tun = dict(tile_qubits=k, reg_qubits=R, fusion_depth=int(rng.integers(0, 7)),
               epoch_fill=int(rng.choice([-1, 0, 1, 2, 3])), uncompute=int(rng.integers(0, 2)),
               ckpt_interval=int(rng.integers(0, 4)), micro_batch=int(rng.integers(0, x.shape[0] + 1)))
    xm, zm = z_observables(obs)
    dE = rng.normal(size=(x.shape[0], len(obs))).astype(np.float32)
    E, dth, dx = pc.run(n, gates, theta, x, zm, dE, **tun)
    assert close(E, dth, dx, orc.backward(n, gates, theta, x, xm, zm, dE)), (n, tun)


@pytest.mark.parametrize("seed", range(40))
def test_random_batch(orc, seed):
    rng = np.random.default_rng(5000 + seed)
    circs, samples, thetas, xs, dEs, refs = [], [], [], [], [], []
    for i in range(int(rng.integers(1, 7))):
        n, gates, theta, x, obs = random_circuit(rng, 10 * seed + i)
        xm, zm = z_observables(obs)
        dE = rng.normal(size=(x.shape[0], len(obs))).astype(np.float32)
        circs.append((n, gates, len(theta), n, zm))
        samples.append(x.shape[0])
        thetas.append(theta)
        xs.append(x)
        dEs.append(dE)
        refs.append(orc.backward(n, gates, theta, x, xm, zm, dE))
    tun = dict(fusion_depth=int(rng.integers(0, 7)), epoch_fill=int(rng.choice([-1, 0, 2])),
               uncompute=int(rng.integers(0, 2)), tile_qubits=int(rng.choice([0, 0, 5, 6, 8])))
    Es, dths, dxs, _ = pc.batch_run(circs, samples, thetas, xs, dEs, **tun)
    for i, ref in enumerate(refs):
        assert close(Es[i], dths[i], dxs[i], ref), (i, circs[i][0], tun)
