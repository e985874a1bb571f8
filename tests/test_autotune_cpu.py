"""Host logic of the autotuner: cache keys and round trip, tuning records, and
the checkpoint choice against a brute-force minimum of the workspace model."""
import json

import numpy as np

from paper_2603_02804_amd import autotune
from paper_2603_02804_amd.workloads import hea_gates


def test_cache_roundtrip(tmp_path):
    g = hea_gates(6, 3, ("RY", "RZ"))
    key = autotune.circuit_key(6, g, 1, 8, "dev")
    assert key == autotune.circuit_key(6, g.copy(), 1, 8, "dev")
    assert key != autotune.circuit_key(6, hea_gates(6, 4, ("RY", "RZ")), 1, 8, "dev")
    assert key != autotune.circuit_key(6, g, 1, 16, "dev")
    path = tmp_path / "tuned.json"
    rec = {"tile_qubits": 12, "reg_qubits": 4, "fusion_depth": 8, "micro_batch": 16, "ckpt_interval": 5,
           "store_ckpt": 1}
    path.write_text(json.dumps({key: rec}))
    assert autotune.cached_tuning(6, g, 1, 8, "dev", path=str(path)) == rec
    assert autotune.cached_tuning(6, g, 1, 8, "other", path=str(path)) is None


def test_tuning_from_fields():
    t = autotune.tuning_from({"tile_qubits": 11, "reg_qubits": 4, "fusion_depth": 12, "micro_batch": 32,
                              "ckpt_interval": 7, "store_ckpt": 0})
    assert (t.mode, t.tile_qubits, t.reg_qubits, t.fusion_depth, t.micro_batch, t.ckpt_interval, t.store_ckpt) == \
        (0, 11, 4, 12, 32, 7, 0)


def test_optimal_ckpt_brute_force():
    for passes, batch, mb, store in [(249, 1000, 16, True), (249, 1000, 16, False), (40, 64, 8, True),
                                     (7, 4, 4, True), (1, 1, 1, True)]:
        c = autotune.optimal_ckpt(passes, batch, mb, store)
        brute = min(autotune.plan_states(passes, k, batch, mb, store) for k in range(1, passes + 1))
        assert autotune.plan_states(passes, c, batch, mb, store) == brute


def test_optimal_ckpt_brute_force_mem_save():
    for passes, batch, mb, store in [(249, 1000, 32, True), (249, 1000, 32, False), (26, 64, 8, True)]:
        c = autotune.optimal_ckpt(passes, batch, mb, store, True)
        brute = min(autotune.plan_states(passes, k, batch, mb, store, True) for k in range(1, passes + 1))
        assert autotune.plan_states(passes, c, batch, mb, store, True) == brute


def test_mem_save_halves_stored_outputs_only():
    # checkpoints and ping-pong states stay full size; the segment's stored outputs halve
    full = autotune.plan_states(100, 10, 64, 8, True, False)
    half = autotune.plan_states(100, 10, 64, 8, True, True)
    assert full - half == 9 * 8 / 2


def test_choose_storage_order():
    S = 8 << 20
    P, B, mb = 249, 1000, 32
    c1 = autotune.optimal_ckpt(P, B, mb, True, False)
    need_full = autotune.plan_states(P, c1, B, mb, True, False) * S
    assert autotune.choose_storage(P, B, mb, S, need_full)[:2] == (1, 0)
    c2 = autotune.optimal_ckpt(P, B, mb, True, True)
    need_half = autotune.plan_states(P, c2, B, mb, True, True) * S
    assert need_half < need_full
    assert autotune.choose_storage(P, B, mb, S, need_half)[:2] == (1, 1)
    assert autotune.choose_storage(P, B, mb, S, 1)[:2] == (0, 1)


def test_tuning_from_mem_save():
    t = autotune.tuning_from({"tile_qubits": 12, "mem_save": 1})
    assert t.mem_save == 1 and t.mode == 0


def test_tuning_from_uncompute_and_fill():
    t = autotune.tuning_from({"uncompute": 1, "epoch_fill": -1, "ckpt_interval": 64})
    assert (t.uncompute, t.epoch_fill, t.ckpt_interval, t.mem_save) == (1, -1, 64, 0)
    t = autotune.tuning_from({})
    assert (t.uncompute, t.epoch_fill) == (0, 0)


def test_uncompute_storage():
    """Uncompute mode: no stored pass outputs, so the workspace is the checkpoints plus four
    micro-batch states; segments of at most UNCOMPUTE_MAX_SEGMENT passes when they fit."""
    SB = 8 << 20
    assert autotune.plan_states(253, 64, 1000, 128, True, False, True) == 4 * 1000 + 4 * 128
    store, c = autotune.uncompute_storage(253, 1000, 128, SB, 200e9)
    assert (store, c) == (1, autotune.UNCOMPUTE_MAX_SEGMENT)
    # a tight budget: fewer, longer segments until the checkpoints fit
    store, c = autotune.uncompute_storage(253, 1000, 128, SB, 3 * 1000 * SB + 4 * 128 * SB)
    assert store == 1 and -(-253 // c) == 3
    # not even one checkpoint of the whole batch fits: checkpoints per micro-batch
    store, c = autotune.uncompute_storage(253, 1000, 128, SB, 1100 * SB)
    assert store == 0 and c == autotune.UNCOMPUTE_MAX_SEGMENT
