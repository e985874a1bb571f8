"""Given initial states on the GPU (fused, per gate, complex128, autograd)
against the oracle started from the same states: the paper's random-state
experiment shape (Sec. 4) with the (IXYZ) observable and a CZ ring."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import paper_mode  # noqa: E402

pytestmark = pytest.mark.gpu
E_TOL, G_TOL = 1e-4, 1e-3


def rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,L,B,tun", [
    (14, 4, 3, {}),
    (16, 3, 2, dict(store_ckpt=0, ckpt_interval=2, micro_batch=1)),
    (20, 2, 2, {}),
    (10, 4, 2, dict(mode=1)),
    (15, 4, 2, dict(uncompute=1, ckpt_interval=2)),
])
def test_paper_mode_against_oracle(n, L, B, tun):
    dev = torch.device("cuda:0")
    w = paper_mode(n, L, B, seed=n)
    circ = qfuse.Circuit(n, w.gates, len(w.theta), 0, w.zmask, w.xmask)
    plan = qfuse.Plan(circ, B, qfuse.make_tuning(**tun) if tun else None)
    ws = plan.new_workspace(dev)
    th = torch.tensor(w.theta, device=dev)
    psi0 = torch.tensor(w.psi0, device=dev)
    dE = np.random.default_rng(n).normal(size=(B, 1)).astype(np.float32)
    E = plan.forward(th, None, ws, psi0=psi0)
    dth, _ = plan.backward(th, None, torch.tensor(dE, device=dev), ws, psi0=psi0)
    torch.cuda.synchronize()
    x = np.zeros((B, 0))
    Eo, dtho, _ = Oracle().backward(n, w.gates, w.theta, x, w.xmask, w.zmask, dE, psi0=w.psi0)
    assert np.abs(E.cpu().numpy() - Eo).max() <= E_TOL
    assert rel(dth.cpu().numpy(), dtho) <= G_TOL


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,B", [(4, 64), (5, 33), (8, 16), (12, 8), (13, 4)])
def test_hea_d1_sweep_shapes_against_oracle(n, B):
    """The one-layer HEA of the throughput sweep (RX, RY, RZ + CZ ring from random states, (IXYZ)...,
    L = sum E) in the plan the benchmark uses (adjoint passes rebuild psi), fused and per gate."""
    dev = torch.device("cuda:0")
    w = paper_mode(n, 1, B, seed=100 + n)
    circ = qfuse.Circuit(n, w.gates, len(w.theta), 0, w.zmask, w.xmask)
    th = torch.tensor(w.theta, device=dev)
    psi0 = torch.tensor(w.psi0, device=dev)
    dE = torch.ones(B, 1, device=dev)
    Eo, dtho, _ = Oracle().backward(n, w.gates, w.theta, np.zeros((B, 0)), w.xmask, w.zmask, np.ones((B, 1)),
                                    psi0=w.psi0)
    for tun in (qfuse.make_tuning(uncompute=1), qfuse.make_tuning(mode=1, micro_batch=B)):
        plan = qfuse.Plan(circ, B, tun)
        ws = plan.new_workspace(dev)
        E = plan.forward(th, None, ws, psi0=psi0)
        dth, _ = plan.backward(th, None, dE, ws, psi0=psi0)
        torch.cuda.synchronize()
        assert np.abs(E.cpu().numpy() - Eo).max() <= E_TOL
        assert rel(dth.cpu().numpy(), dtho) <= G_TOL


def test_paper_mode_c128_gradcheck():
    dev = torch.device("cuda:0")
    n, L, B = 4, 2, 2
    w = paper_mode(n, L, B, seed=2)
    circ = qfuse.Circuit(n, w.gates, len(w.theta), 0, w.zmask, w.xmask)
    plan = qfuse.Plan(circ, B, qfuse.make_tuning(mode=qfuse.QF_MODE_C128))
    psi0 = torch.tensor(w.psi0.astype(np.complex128), device=dev)
    theta = torch.tensor(w.theta.astype(np.float64), device=dev, requires_grad=True)
    E = qfuse.circuit_expectations(theta, None, plan, psi0=psi0)
    Eo = Oracle().forward(n, w.gates, w.theta.astype(np.float64), np.zeros((B, 0)), w.xmask, w.zmask,
                          psi0=w.psi0.astype(np.complex128))
    assert np.abs(E.detach().cpu().numpy() - Eo).max() <= 1e-10
    assert torch.autograd.gradcheck(lambda t: qfuse.circuit_expectations(t, None, plan, True, psi0), (theta,),
                                    eps=1e-6, atol=1e-7, rtol=1e-5)


def test_psi0_shape_checked():
    dev = torch.device("cuda:0")
    w = paper_mode(6, 1, 2, seed=1)
    plan = qfuse.Plan(qfuse.Circuit(6, w.gates, len(w.theta), 0, w.zmask, w.xmask), 2)
    ws = plan.new_workspace(dev)
    th = torch.tensor(w.theta, device=dev)
    with pytest.raises(ValueError):
        plan.forward(th, None, ws, psi0=torch.zeros(2, 32, dtype=torch.complex64, device=dev))
