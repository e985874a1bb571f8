"""qf_forward_noalloc (the forward for callers that cannot allocate) against
qf_forward with a caller workspace: same plan, same inputs, two calls in a row
on the library's shared device array, the second with a smaller circuit and
batch, both checked bit for bit against qf_forward and within the float32
tolerance against the complex128 oracle (expectations of Sec. 2.1).  A plan
whose workspace exceeds the array is refused with QF_ERR_WORKSPACE.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import draw_inputs, hea_gates, z_observables  # noqa: E402

pytestmark = pytest.mark.gpu

E_TOL = 1e-4
SCRATCH_BYTES = 64 << 20


def _case(n, L, B, seed, obs, uncompute):
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    theta, x, _ = draw_inputs(seed, L * 3 * n, B, n)
    xm, zm = z_observables(obs)
    circ = qfuse.Circuit(n, gates, len(theta), n, zm)
    plan = qfuse.Plan(circ, B, qfuse.make_tuning(uncompute=uncompute, ckpt_interval=2))
    return gates, theta, x, xm, zm, plan


def test_noalloc_matches_forward_twice_then_smaller():
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    orc = Oracle()
    # first a multi-tile circuit, then a smaller one: the second call reuses the
    # array the first left behind
    for n, L, B, seed, obs, unc in ((14, 3, 4, 11, [0, 5, 13], 1), (9, 4, 2, 12, [0, 8], 0)):
        gates, theta, x, xm, zm, plan = _case(n, L, B, seed, obs, unc)
        assert plan.ws_bytes <= SCRATCH_BYTES
        print(f"noalloc case n={n} L={L} B={B} ws={plan.ws_bytes}", flush=True)
        th, xx = torch.tensor(theta, device=dev), torch.tensor(x, device=dev)
        ws = plan.new_workspace(dev)
        E_ref = plan.forward(th, xx, ws)
        E_na = plan.forward_noalloc(th, xx)
        E_na2 = plan.forward_noalloc(th, xx)
        torch.cuda.synchronize()
        a, b, b2 = E_ref.cpu().numpy(), E_na.cpu().numpy(), E_na2.cpu().numpy()
        assert np.array_equal(a, b), f"noalloc differs from qf_forward: {np.abs(a - b).max():.3e}"
        assert np.array_equal(a, b2)
        Eo = orc.forward(n, gates, theta, x, xm, zm)
        assert np.abs(b - Eo).max() <= E_TOL, f"E err {np.abs(b - Eo).max():.3e}"


def test_noalloc_refuses_a_plan_beyond_the_array():
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, B = 20, 8
    gates = hea_gates(n, 1, ("RY",))
    theta, x, _ = draw_inputs(1, n, B, n)
    xm, zm = z_observables([0])
    plan = qfuse.Plan(qfuse.Circuit(n, gates, len(theta), n, zm), B)
    assert plan.ws_bytes > SCRATCH_BYTES
    th, xx = torch.tensor(theta, device=dev), torch.tensor(x, device=dev)
    with pytest.raises(qfuse.QFuseError) as ei:
        plan.forward_noalloc(th, xx)
    assert ei.value.status == 3 and "qf_forward_noalloc" in str(ei.value)
