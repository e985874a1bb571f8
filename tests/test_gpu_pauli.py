"""General Pauli-string observables on the GPU (fused, per gate, complex128)
against the oracle, and their rejection by mixed batches."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import draw_inputs, hea_gates, pauli_string  # noqa: E402
from pauli_cases import strings  # noqa: E402

pytestmark = pytest.mark.gpu
E_TOL, G_TOL = 1e-4, 1e-3


def rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


def _run(n, gates, theta, x, xm, zm, dE, dtype=torch.float32, **tun):
    dev = torch.device("cuda:0")
    circ = qfuse.Circuit(n, gates, len(theta), x.shape[1], zm, xm)
    plan = qfuse.Plan(circ, x.shape[0], qfuse.make_tuning(**tun) if tun else None)
    ws = plan.new_workspace(dev)
    th = torch.tensor(theta, dtype=dtype, device=dev)
    xx = torch.tensor(x, dtype=dtype, device=dev)
    E = plan.forward(th, xx, ws)
    dth, dx = plan.backward(th, xx, torch.tensor(dE, dtype=dtype, device=dev), ws)
    torch.cuda.synchronize()
    return E.cpu().numpy(), dth.cpu().numpy(), dx.cpu().numpy()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,L,B,tun", [
    (14, 4, 3, {}),
    (16, 3, 2, dict(ckpt_interval=2, micro_batch=1)),
    (20, 2, 2, {}),
    (12, 5, 2, dict(tile_qubits=11, reg_qubits=4)),
    (9, 6, 4, {}),
    (14, 3, 2, dict(mode=1)),
    (15, 4, 2, dict(uncompute=1, ckpt_interval=2)),
])
def test_pauli_against_oracle(n, L, B, tun):
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    theta, x, _ = draw_inputs(90 + n, L * 3 * n, B, n)
    xm, zm = strings(n)
    dE = np.random.default_rng(n).normal(size=(B, len(zm))).astype(np.float32)
    E, dth, dx = _run(n, gates, theta, x, xm, zm, dE, **tun)
    Eo, dtho, dxo = Oracle().backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL
    assert rel(dth, dtho) <= G_TOL and rel(dx, dxo) <= G_TOL


def test_pauli_c128_exact():
    n, L, B = 8, 3, 2
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    rng = np.random.default_rng(8)
    theta = rng.uniform(-3, 3, L * 3 * n)
    x = rng.uniform(-3, 3, (B, n))
    xm, zm = strings(n)
    dE = rng.normal(size=(B, len(zm)))
    E, dth, dx = _run(n, gates, theta, x, xm, zm, dE, dtype=torch.float64, mode=qfuse.QF_MODE_C128)
    Eo, dtho, dxo = Oracle().backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= 1e-10
    assert rel(dth, dtho) <= 1e-9 and rel(dx, dxo) <= 1e-9


def test_mixed_batch_rejects_x_and_y():
    gates = hea_gates(5, 2, ("RY", "RZ"))
    xm, zm = pauli_string("IIIIX")
    c1 = qfuse.Circuit(5, gates, 20, 5, [0], [xm])
    c2 = qfuse.Circuit(5, gates, 20, 5, [1])
    with pytest.raises(qfuse.QFuseError) as e:
        qfuse.Batch([c2, c1], [1, 1])
    assert e.value.status == 2
