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
from paper_2603_02804_amd.workloads import z_observables
from random_cases import close, random_batch_tuning, random_circuit, random_tuning, random_tuning_wide


@pytest.fixture(scope="module")
def orc():
    return Oracle()


@pytest.mark.parametrize("seed", range(200))
def test_random_plan(orc, seed):
    rng = np.random.default_rng(1000 + seed)
    n, gates, theta, x, obs = random_circuit(rng, seed)
    tun = random_tuning(rng, n, x.shape[0])
    xm, zm = z_observables(obs)
    dE = rng.normal(size=(x.shape[0], len(obs))).astype(np.float32)
    E, dth, dx = pc.run(n, gates, theta, x, zm, dE, **tun)
    assert close(E, dth, dx, orc.backward(n, gates, theta, x, xm, zm, dE)), (n, tun)


@pytest.mark.parametrize("seed", range(30))
def test_random_wide_plan(orc, seed):
    rng = np.random.default_rng(9000 + seed)
    n = 0
    while n < 10:
        n, gates, theta, x, obs = random_circuit(rng, seed, max_n=16)
    tun = random_tuning_wide(rng, n, x.shape[0])
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
    tun = random_batch_tuning(rng)
    Es, dths, dxs, _ = pc.batch_run(circs, samples, thetas, xs, dEs, **tun)
    for i, ref in enumerate(refs):
        assert close(Es[i], dths[i], dxs[i], ref), (i, circs[i][0], tun)
