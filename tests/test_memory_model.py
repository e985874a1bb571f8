"""The memory model against the paper's printed values, and the planner's
workspace against its closed form."""
import json
import math
import os

import pytest

import plancheck as pc
from paper_2603_02804_amd.autotune import optimal_ckpt, paper_memory_bytes, paper_optimal_block, plan_states
from paper_2603_02804_amd.workloads import hea_gates

FIX = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_memory_model.json")))


@pytest.mark.parametrize("case", FIX["cases"], ids=lambda c: c["what"])
def test_paper_measured_memory(case):
    """(s b + d/b) M_sv reproduces the printed peak memory within 5 percent (Sec. 4.3.1)."""
    m = paper_memory_bytes(case["stored_per_layer"], case["d"], case["b"], FIX["m_sv_bytes"])
    assert abs(m / 1e6 - case["measured_MB"]) / case["measured_MB"] <= 0.05


@pytest.mark.parametrize("case", FIX["optimal_b"], ids=lambda c: c["what"])
def test_paper_optimal_block(case):
    """b* = sqrt(d / s) as printed (Sec. 4.3.1, App. C), to the printed precision."""
    b = paper_optimal_block(case["stored_per_layer"], case["d"])
    tol = 0.5 if case["printed_digits"] == 0 else 0.1
    assert abs(b - case["printed"]) <= tol


def test_model_minimum_is_sqrt():
    """The memory model's minimum over b sits at sqrt(d/s) and equals 2 sqrt(s d) M_sv."""
    s, d = 7, 1000
    best = min(range(1, 200), key=lambda b: paper_memory_bytes(s, d, b, 1))
    assert abs(best - paper_optimal_block(s, d)) < 1
    assert paper_memory_bytes(s, d, math.sqrt(d / s), 1) == pytest.approx(2 * math.sqrt(s * d))


def test_planner_workspace_matches_closed_form():
    """Checkpoint and pass-output storage of the plan follow plan_states()."""
    n, L, B = 14, 12, 8
    g = hea_gates(n, L, ("RX", "RY", "RZ"))
    for ckpt, mb in ((2, 2), (3, 4), (5, 8)):
        st = pc.stats(n, g, L * 3 * n, n, [1], B, ckpt_interval=ckpt, micro_batch=mb)
        states = plan_states(st["passes"], st["ckpt"], B, st["micro_batch"], True)
        S = 8 << n
        # the workspace holds these states plus small tables and partial sums
        assert states * S <= st["ws_bytes"] <= states * S + (4 << 20)


def test_optimal_ckpt_minimises_states():
    P, B, mb = 250, 1000, 16
    c = optimal_ckpt(P, B, mb)
    assert all(plan_states(P, c, B, mb) <= plan_states(P, c2, B, mb) for c2 in range(1, P + 1))
