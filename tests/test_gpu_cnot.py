"""CNOT gates on the GPU (fused, per gate, complex128) against the oracle's
textbook CNOT: ladders and rings between the rotation layers."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import CNOT, draw_inputs, hea_gates  # noqa: E402
from pauli_cases import strings  # noqa: E402

pytestmark = pytest.mark.gpu
E_TOL, G_TOL = 1e-4, 1e-3


def rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,L,ring,dtype,tun", [
    (14, 4, False, torch.float32, {}),
    (16, 3, True, torch.float32, dict(ckpt_interval=2, micro_batch=1)),
    (20, 2, False, torch.float32, {}),
    (10, 3, True, torch.float32, dict(mode=1)),
    (7, 3, True, torch.float64, dict(mode=2)),
])
def test_cnot_against_oracle(n, L, ring, dtype, tun):
    dev = torch.device("cuda:0")
    gates = hea_gates(n, L, ("RX", "RY", "RZ"), ring=ring, entangler=CNOT)
    theta, x, _ = draw_inputs(130 + n, L * 3 * n, 2, n)
    xm, zm = strings(n)
    dE = np.random.default_rng(n).normal(size=(2, len(zm)))
    circ = qfuse.Circuit(n, gates, len(theta), n, zm, xm)
    plan = qfuse.Plan(circ, 2, qfuse.make_tuning(**tun) if tun else None)
    ws = plan.new_workspace(dev)
    th = torch.tensor(theta, dtype=dtype, device=dev)
    xx = torch.tensor(x, dtype=dtype, device=dev)
    E = plan.forward(th, xx, ws)
    dth, dx = plan.backward(th, xx, torch.tensor(dE, dtype=dtype, device=dev), ws)
    torch.cuda.synchronize()
    Eo, dtho, dxo = Oracle().backward(n, gates, theta, x, xm, zm, dE)
    etol, gtol = (1e-10, 1e-9) if dtype == torch.float64 else (E_TOL, G_TOL)
    assert np.abs(E.cpu().numpy() - Eo).max() <= etol
    assert rel(dth.cpu().numpy(), dtho) <= gtol and rel(dx.cpu().numpy(), dxo) <= gtol
