"""Planner and driver on the CPU: the fused programs, executed thread by thread by
the test-only schedule checker (with bounds assertions on every LDS, state and
partial-sum access), agree with the oracle for every configuration the GPU parity
tests launch, and the schedules satisfy their structural invariants."""
import numpy as np
import pytest

import plancheck as pc
from oracle.oracle import Oracle
from paper_2603_02804_amd.workloads import CZ, RX, RY, draw_inputs, hea_gates, z_observables

E_TOL = 1e-4
G_TOL = 1e-3

SINGLE = [
    (1, 3, ("RX", "RY", "RZ"), 3, {}),
    (5, 3, ("RY", "RZ"), 5, {}),
    (7, 4, ("RX", "RY", "RZ"), 3, {"fusion_depth": 2}),
    (10, 3, ("RY", "RZ"), 4, {}),
    (11, 3, ("RX", "RY", "RZ"), 3, {"fusion_depth": 1, "ckpt_interval": 2}),
    (12, 5, ("RY", "RZ"), 6, {}),
    (13, 3, ("RX", "RY", "RZ"), 2, {}),
]
MULTI = [
    (9, 4, ("RY", "RZ"), 3, {"tile_qubits": 7, "reg_qubits": 2}),
    (10, 5, ("RX", "RY", "RZ"), 3, {"tile_qubits": 8, "reg_qubits": 4, "ckpt_interval": 2, "micro_batch": 2}),
    (12, 4, ("RX", "RY", "RZ"), 5, {"tile_qubits": 11, "fusion_depth": 2, "ckpt_interval": 3, "micro_batch": 2}),
    (14, 3, ("RX", "RY", "RZ"), 3, {}),
    (15, 4, ("RY", "RZ"), 2, {"store_ckpt": 0, "micro_batch": 1}),
    (16, 3, ("RX", "RY", "RZ"), 2, {"fusion_depth": 8}),
    (14, 6, ("RY", "RZ"), 2, {"fusion_depth": 12}),   # epochs with up to 3 register-bit phases
]


@pytest.fixture(scope="module")
def orc():
    return Oracle()


def rel(a, b):
    s = float(np.abs(b).max()) if np.size(b) else 0.0
    d = float(np.abs(np.asarray(a, np.float64) - b).max()) if np.size(b) else 0.0
    return d / s if s > 0 else d


def check(orc, n, gates, theta, x, obs, seed=0, **tun):
    xm, zm = z_observables(obs)
    dE = np.random.default_rng(seed).normal(size=(x.shape[0], len(obs))).astype(np.float32)
    E, dth, dx = pc.run(n, gates, theta, x, zm, dE, **tun)
    Eo, dtho, dxo = orc.backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL
    assert rel(dth, dtho) <= G_TOL
    if x.shape[1]:
        assert rel(dx, dxo) <= G_TOL


@pytest.mark.parametrize("n,L,rots,B,tun", SINGLE + MULTI)
def test_hea_programs(orc, n, L, rots, B, tun):
    gates = hea_gates(n, L, rots)
    theta, x, _ = draw_inputs(21, L * len(rots) * n, B, n)
    obs = [0, n - 1] if n > 1 else [0]
    if (n, L, rots, B, tun) in MULTI:
        obs = [0, 3, n - 1]
    check(orc, n, gates, theta, x, obs, **tun)


@pytest.mark.parametrize("k,R", [(1, 1), (2, 1), (2, 2), (3, 2), (4, 3), (4, 4), (5, 4)])
def test_small_tiles(orc, k, R):
    """Tiles of a few qubits on a wider register (each pass brings in at least one
    new qubit next to the ones kept at the lowest memory bits) against the oracle."""
    n, L, B = 7, 3, 2
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    theta, x, _ = draw_inputs(31, L * 3 * n, B, n)
    check(orc, n, gates, theta, x, [0, 3, n - 1], tile_qubits=k, reg_qubits=R, fusion_depth=2)


@pytest.mark.parametrize("tun", [{}, {"tile_qubits": 8, "reg_qubits": 3, "fusion_depth": 2}, {"mode": 1}])
def test_general_gate_list(orc, tun):
    rng = np.random.default_rng(5)
    n, B = 11, 3
    rows = [(RY, q, -1, -1, q) for q in range(n)]
    for _ in range(120):
        k = int(rng.integers(0, 4))
        q0 = int(rng.integers(0, n))
        if k == CZ:
            rows.append((CZ, q0, int((q0 + 1 + rng.integers(0, n - 1)) % n), -1, -1))
        elif rng.random() < 0.15:
            rows.append((k, q0, -1, -1, int(rng.integers(0, n))))
        else:
            rows.append((k, q0, -1, int(rng.integers(0, 40)), -1))
    gates = np.asarray(rows, dtype=np.int32)
    theta, x, _ = draw_inputs(9, 40, B, n)
    check(orc, n, gates, theta, x, [0, 5, 10], **tun)


def test_ring(orc):
    gates = hea_gates(9, 3, ("RX", "RY", "RZ"), ring=True)
    theta, x, _ = draw_inputs(3, 81, 4, 9)
    check(orc, 9, gates, theta, x, [0, 4, 8], tile_qubits=7, reg_qubits=3)


@pytest.mark.parametrize("n,L", [(6, 3), (11, 3)])
def test_per_gate_programs(orc, n, L):
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    theta, x, _ = draw_inputs(21, L * 3 * n, 3, n)
    check(orc, n, gates, theta, x, [0, 2], mode=1)


def test_schedule_shape_at_benchmark_sizes():
    """20 qubits x 1000 layers: tiles of 2^12 amplitudes, register blocks of 4
    qubits and several layers fused per HBM round trip."""
    g = hea_gates(20, 1000, ("RX", "RY", "RZ"))
    st = pc.stats(20, g, 60000, 20, [1], 1000, fusion_depth=8)
    assert st["k"] == 12 and st["R"] == 4
    assert st["runs"] == 20 * 1000          # encoding merged into layer 1
    assert st["u2"] == st["runs"]           # every run applied exactly once
    assert st["passes"] < 1000              # more than one layer per pass on average


@pytest.mark.parametrize("n", [3, 6, 9, 10, 11, 12, 13, 16])
def test_wide_workgroups_cover_whole_tiles(n):
    """Workgroups of more than one wave hold exactly the tile's threads (the adjoint
    pass drops the functionals of idle lanes only in 64-thread workgroups)."""
    g = hea_gates(n, 2, ("RY", "RZ"))
    for k in range(1, min(n, 13) + 1):
        for R in range(1, min(k, 5) + 1):
            if k - R > 8:
                continue
            st = pc.stats(n, g, 2 * 2 * n, n, [1], 4, tile_qubits=k, reg_qubits=R)
            assert st["threads"] in (64, 1 << st["thread_bits"]), (n, k, R, st)
            assert st["threads"] >= 1 << st["thread_bits"]


@pytest.mark.parametrize("fill", [-1, 1, 2, 0])
def test_epoch_fill_programs(orc, fill):
    """Every end-of-pass epoch threshold gives the same results (a ring, so that
    partial epochs at pass ends are common)."""
    gates = hea_gates(14, 5, ("RX", "RY", "RZ"), ring=True)
    theta, x, _ = draw_inputs(31, 5 * 3 * 14, 2, 14)
    check(orc, 14, gates, theta, x, [0, 7, 13], epoch_fill=fill)


def test_epoch_fill_trades_epochs_for_passes():
    """Leaving partial end-of-pass epochs to the next pass: no more register
    epochs (PERMs), and on a CZ ring far fewer, for at most a few more passes."""
    g = hea_gates(20, 60, ("RX", "RY", "RZ"), encoding=False, ring=True)
    off = pc.stats(20, g, 3600, 0, [1], 8, epoch_fill=-1)
    on = pc.stats(20, g, 3600, 0, [1], 8)
    assert on["u2"] == off["u2"] == 20 * 60
    assert on["perm"] < 0.97 * off["perm"]   # (exchanges within passes: loads and stores need none)
    assert on["passes"] < off["passes"]
    g = hea_gates(20, 60, ("RX", "RY", "RZ"))
    off = pc.stats(20, g, 3600, 20, [1], 8, epoch_fill=-1)
    on = pc.stats(20, g, 3600, 20, [1], 8)
    assert on["perm"] <= off["perm"] and on["passes"] <= off["passes"] + 2


@pytest.mark.parametrize("n,L,rots,B,tun", [
    (13, 3, ("RX", "RY", "RZ"), 2, {}),
    (14, 4, ("RX", "RY", "RZ"), 3, {"ckpt_interval": 2, "micro_batch": 2}),
    (15, 4, ("RY", "RZ"), 2, {"store_ckpt": 0, "micro_batch": 1}),
    (12, 5, ("RX", "RY", "RZ"), 4, {"tile_qubits": 8, "reg_qubits": 3, "fusion_depth": 2}),
    (10, 5, ("RX", "RY", "RZ"), 3, {"tile_qubits": 8, "reg_qubits": 4, "ckpt_interval": 2, "micro_batch": 2}),
])
def test_uncompute_programs(orc, n, L, rots, B, tun):
    """The adjoint passes write psi at their input, so the backward recomputes
    nothing; results match the oracle (and the recompute scheme)."""
    gates = hea_gates(n, L, rots)
    theta, x, _ = draw_inputs(41, L * len(rots) * n, B, n)
    check(orc, n, gates, theta, x, [0, 3, n - 1], uncompute=1, **tun)


def test_uncompute_drift_over_one_long_segment(orc):
    """psi rebuilt through 16 fused passes (60 layers, one checkpoint segment):
    the float32 drift of the reconstruction stays far inside the tolerance."""
    n, L, B = 14, 60, 2
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    theta, x, _ = draw_inputs(8, L * 3 * n, B, n)
    xm, zm = z_observables([0, 3, n - 1])
    dE = np.random.default_rng(1).normal(size=(B, 3)).astype(np.float32)
    Eo, dtho, dxo = orc.backward(n, gates, theta, x, xm, zm, dE)
    st = pc.stats(n, gates, len(theta), n, zm, B, uncompute=1, ckpt_interval=1000)
    assert st["segments"] == 1 and st["passes"] > 10
    E, dth, dx = pc.run(n, gates, theta, x, zm, dE, uncompute=1, ckpt_interval=1000)
    assert np.linalg.norm(dth - dtho) / np.linalg.norm(dtho) <= 1e-4
    assert np.linalg.norm(dx - dxo) / np.linalg.norm(dxo) <= 1e-4


def test_uncompute_workspace_holds_no_segment_states():
    g = hea_gates(16, 40, ("RX", "RY", "RZ"))
    rec = pc.stats(16, g, 40 * 48, 16, [1], 8, ckpt_interval=4, micro_batch=4)
    unc = pc.stats(16, g, 40 * 48, 16, [1], 8, ckpt_interval=4, micro_batch=4, uncompute=1)
    SB = 8 << 16
    assert rec["ws_bytes"] - unc["ws_bytes"] >= 3 * 4 * SB   # (ckpt - 1) x micro-batch stored outputs


@pytest.mark.parametrize("n,L,rots,tun", [
    (20, 64, ("RX", "RY", "RZ"), {"fusion_depth": 4, "uncompute": 1}),
    (20, 64, ("RX", "RY", "RZ"), {"fusion_depth": 8}),
    (16, 40, ("RX", "RY", "RZ"), {"fusion_depth": 16, "uncompute": 1}),
    (13, 30, ("RY", "RZ"), {"fusion_depth": 12, "uncompute": 1, "epoch_fill": -1}),
    (18, 30, ("RY", "RZ"), {"fusion_depth": 12, "uncompute": 1, "epoch_fill": -1}),
    (12, 30, ("RY", "RZ"), {"fusion_depth": 12}),
    (11, 20, ("RY", "RZ"), {"fusion_depth": 12}),
])
def test_exchanges_free_of_lds_bank_conflicts(n, L, rots, tun):
    """Tiles of 11 and 12 qubits: in every exchange layout the 32 lanes of one LDS
    cycle place their 8-byte elements in 32 distinct bank slots (the swizzle folds
    tile bits 5 and up onto element bits 0..4 and the planner orders lanes 0..4 to be
    independent there)."""
    g = hea_gates(n, L, rots)
    st = pc.stats(n, g, len(rots) * n * L, n, [1], 4, **tun)
    assert st["k"] >= 11 and st["lds_bank_degree"] == 1, st


def test_ten_qubit_tiles_share_at_most_two_elements_per_bank_slot():
    """Tiles of 10 qubits (64 threads) cannot be conflict-free for every choice of
    register positions under one fixed fold set; they stay at two elements per slot."""
    g = hea_gates(10, 20, ("RY", "RZ"))
    st = pc.stats(10, g, 400, 10, [1], 4, fusion_depth=12)
    assert st["k"] == 10 and st["lds_bank_degree"] <= 2, st
