"""Mixed batches on the CPU checker: the merged launch sequences, replayed job by
job with the emulated kernels, give exactly the results of each circuit alone,
and match the oracle.  Also the launch accounting of the merge."""
import numpy as np
import pytest

import plancheck
from oracle.oracle import Oracle
from paper_2603_02804_amd.workloads import mixed, z_observables


def _circuits(ws):
    xm, zm = z_observables([0])
    return [(c.n_qubits, c.gates, len(c.theta), c.n_qubits, zm) for c in ws], zm


def _dEs(ws, seed):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=(c.x.shape[0], 1)).astype(np.float32) for c in ws]


@pytest.mark.parametrize("case", [
    dict(n=6, qubits=(3, 9), layers=(1, 6), samples=3, seed=11, tuning={}),
    dict(n=5, qubits=(11, 14), layers=(2, 5), samples=2, seed=12, tuning=dict(fusion_depth=2, ckpt_interval=2)),
    dict(n=4, qubits=(12, 13), layers=(3, 6), samples=5, seed=13, tuning=dict(micro_batch=2, ckpt_interval=3)),
    dict(n=4, qubits=(12, 14), layers=(4, 8), samples=3, seed=14, tuning=dict(ckpt_interval=2, mem_save=1)),
    dict(n=4, qubits=(13, 15), layers=(4, 7), samples=2, seed=15, tuning=dict(epoch_fill=4)),
    dict(n=5, qubits=(11, 15), layers=(3, 7), samples=2, seed=16, tuning=dict(uncompute=1, ckpt_interval=2)),
])
def test_batch_replay_equals_single(case):
    ws = mixed(case["n"], case["qubits"], case["layers"], case["samples"], case["seed"])
    circuits, zm = _circuits(ws)
    dEs = _dEs(ws, case["seed"])
    samples = [c.x.shape[0] for c in ws]
    Es, dth, dxs, st = plancheck.batch_run(circuits, samples, [c.theta for c in ws], [c.x for c in ws], dEs,
                                           **case["tuning"])
    for i, c in enumerate(ws):
        single = dict(case["tuning"])
        # the defaults of a batch's plans: end-of-pass epochs of fewer than 2 runs wait
        # for the next pass, and fusion depth 12 for circuits larger than one tile
        single.setdefault("epoch_fill", 2)
        if c.n_qubits > single.get("tile_qubits", 12):
            single.setdefault("fusion_depth", 12)
        E1, dth1, dx1 = plancheck.run(c.n_qubits, c.gates, c.theta, c.x, zm, dEs[i], **single)
        np.testing.assert_array_equal(Es[i], E1)
        np.testing.assert_array_equal(dth[i], dth1)
        np.testing.assert_array_equal(dxs[i], dx1)
    assert st["fwd_jobs"] >= st["fwd_launches"] and st["bwd_jobs"] >= st["bwd_launches"]
    assert st["max_jobs_per_launch"] > 1


def test_batch_replay_matches_oracle():
    ws = mixed(5, (4, 13), (2, 4), 2, 21)
    circuits, zm = _circuits(ws)
    xm = np.zeros_like(zm)
    dEs = _dEs(ws, 3)
    Es, dth, dxs, _ = plancheck.batch_run(circuits, [2] * len(ws), [c.theta for c in ws], [c.x for c in ws], dEs)
    orc = Oracle()
    for i, c in enumerate(ws):
        Eo = orc.forward(c.n_qubits, c.gates, c.theta, c.x, xm, zm)
        _, dtho, dxo = orc.backward(c.n_qubits, c.gates, c.theta, c.x, xm, zm, dEs[i].astype(np.float64))
        assert np.abs(Es[i] - Eo).max() <= 1e-4
        assert np.abs(dth[i] - dtho).max() <= 1e-3 * np.abs(dtho).max()
        assert np.abs(dxs[i] - dxo).max() <= 1e-3 * np.abs(dxo).max()


def test_batch_merge_accounting():
    """The merged sequence is as long as the longest circuit's, with one launch per
    kernel variant present at a step."""
    ws = mixed(12, (10, 14), (5, 30), 4, 5)
    circuits, zm = _circuits(ws)
    samples = [4] * len(ws)
    steps = []
    for c in ws:
        s = plancheck.stats(c.n_qubits, c.gates, len(c.theta), c.n_qubits, zm, 4)
        steps.append(s["passes"])
    Es, dth, dxs, st = plancheck.batch_run(circuits, samples, [c.theta for c in ws], [c.x for c in ws], None)
    # forward of one circuit: coefficients, phase events, its passes, the expectation reduction
    assert st["fwd_steps"] <= max(steps) + 3
    assert st["fwd_jobs"] <= sum(p + 3 for p in steps)
    assert st["fwd_launches"] < st["fwd_jobs"] / 2
