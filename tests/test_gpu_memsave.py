"""Memory-saving mode on the GPU (bfloat16 copies of the stored pass outputs):
expectations bit for bit those of the float32 path, gradients within the
rounding bound of bfloat16 storage around the oracle (tests/memsave_bound.py),
mixed batches equal to their circuits' own plans."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from memsave_bound import gradient_bounds, lambda_norms  # noqa: E402
from oracle.oracle import Oracle  # noqa: E402
from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import draw_inputs, hea_gates, mixed, z_observables  # noqa: E402

pytestmark = pytest.mark.gpu
G_TOL = 1e-3


def _run(n, gates, theta, x, zm, dE, **tun):
    dev = torch.device("cuda:0")
    circ = qfuse.Circuit(n, gates, len(theta), x.shape[1], zm)
    plan = qfuse.Plan(circ, x.shape[0], qfuse.make_tuning(**tun))
    ws = plan.new_workspace(dev)
    th = torch.tensor(theta, device=dev)
    xx = torch.tensor(x, device=dev)
    E = plan.forward(th, xx, ws)
    dth, dx = plan.backward(th, xx, torch.tensor(dE, dtype=torch.float32, device=dev), ws)
    torch.cuda.synchronize()
    return E.cpu().numpy(), dth.cpu().numpy(), dx.cpu().numpy(), plan


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,L,B,ckpt,mb", [(16, 10, 3, 2, 2), (20, 12, 2, 2, 2)])
def test_mem_save_against_oracle(n, L, B, ckpt, mb):
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    P = L * 3 * n
    theta, x, _ = draw_inputs(60 + n, P, B, n)
    xm, zm = z_observables([0, n // 2])
    dE = np.random.default_rng(n).normal(size=(B, 2)).astype(np.float32)
    E0, dth0, dx0, p0 = _run(n, gates, theta, x, zm, dE, ckpt_interval=ckpt, micro_batch=mb)
    E1, dth1, dx1, p1 = _run(n, gates, theta, x, zm, dE, ckpt_interval=ckpt, micro_batch=mb, mem_save=1)
    assert p1.info.mem_save == 1 and p1.info.fused_passes > 2   # stored outputs in some segment
    assert p1.ws_bytes < p0.ws_bytes
    np.testing.assert_array_equal(E0, E1)
    orc = Oracle()
    _, dtho, dxo = orc.backward(n, gates, theta, x, xm, zm, dE)
    lam = lambda_norms(orc, n, gates, theta, x, zm, dE)
    bth, bx = gradient_bounds(gates, P, n, lam)
    assert np.all(np.abs(dth1 - dtho) <= bth + G_TOL * np.abs(dtho).max())
    assert np.all(np.abs(dx1 - dxo) <= bx + G_TOL * np.abs(dxo).max())
    assert not np.array_equal(dth0, dth1)


@pytest.mark.timeout(300)
def test_mem_save_mixed_batch_equals_single_plans():
    dev = torch.device("cuda:0")
    ws = mixed(6, (12, 15), (4, 8), 3, 41)
    xm, zm = z_observables([0])
    tun = qfuse.make_tuning(ckpt_interval=2, mem_save=1, epoch_fill=-1)   # a batch's default threshold
    circs = [qfuse.Circuit(c.n_qubits, c.gates, len(c.theta), c.n_qubits, zm) for c in ws]
    thetas = [torch.tensor(c.theta, device=dev) for c in ws]
    xs = [torch.tensor(c.x, device=dev) for c in ws]
    rng = np.random.default_rng(5)
    dEs = [torch.tensor(rng.normal(size=(c.x.shape[0], 1)).astype(np.float32), device=dev) for c in ws]
    batch = qfuse.Batch(circs, [c.x.shape[0] for c in ws], tun)
    wsb = batch.new_workspace(dev)
    Es = batch.forward(thetas, xs, wsb)
    dths, dxs = batch.backward(thetas, xs, dEs, wsb)
    torch.cuda.synchronize()
    for i, (c, w) in enumerate(zip(circs, ws)):
        plan = qfuse.Plan(c, w.x.shape[0], tun)
        wp = plan.new_workspace(dev)
        E = plan.forward(thetas[i], xs[i], wp)
        dth, dx = plan.backward(thetas[i], xs[i], dEs[i], wp)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(Es[i].cpu().numpy(), E.cpu().numpy())
        np.testing.assert_array_equal(dths[i].cpu().numpy(), dth.cpu().numpy())
        np.testing.assert_array_equal(dxs[i].cpu().numpy(), dx.cpu().numpy())
