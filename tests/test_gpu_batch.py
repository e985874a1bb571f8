"""Mixed batches on the GPU: every launch mode gives, for every circuit, exactly
the result of that circuit's own plan (same kernels, same rounding), and the
oracle's within the tolerances; the HIP graph replays stay correct across
replays, new inputs in the same buffers and a new workspace address."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import mixed, z_observables  # noqa: E402

pytestmark = pytest.mark.gpu

MODES = (qfuse.QF_LAUNCH_GRAPH, qfuse.QF_LAUNCH_MERGED, qfuse.QF_LAUNCH_PER_CIRCUIT)


def _setup(ws, dev, seed=0):
    xm, zm = z_observables([0])
    circs = [qfuse.Circuit(c.n_qubits, c.gates, len(c.theta), c.n_qubits, zm) for c in ws]
    thetas = [torch.tensor(c.theta, device=dev) for c in ws]
    xs = [torch.tensor(c.x, device=dev) for c in ws]
    rng = np.random.default_rng(seed)
    dEs = [torch.tensor(rng.normal(size=(c.x.shape[0], 1)).astype(np.float32), device=dev) for c in ws]
    return circs, thetas, xs, dEs, xm, zm


def _single(circs, ws, thetas, xs, dEs, dev, **tun):
    out = []
    for c, w, t, x, d in zip(circs, ws, thetas, xs, dEs):
        # a batch's defaults: end-of-pass epochs of fewer than 2 runs wait, fusion depth 12
        # beyond one tile
        t_c = dict(tun)
        t_c.setdefault("epoch_fill", 2)
        if w.n_qubits > t_c.get("tile_qubits", 12):
            t_c.setdefault("fusion_depth", 12)
        plan = qfuse.Plan(c, w.x.shape[0], qfuse.make_tuning(**t_c))
        wsb = plan.new_workspace(dev)
        E = plan.forward(t, x, wsb)
        dth, dx = plan.backward(t, x, d, wsb)
        out.append((E.cpu().numpy(), dth.cpu().numpy(), dx.cpu().numpy()))
    return out


def _batch(batch, thetas, xs, dEs, wsb):
    Es = batch.forward(thetas, xs, wsb)
    dths, dxs = batch.backward(thetas, xs, dEs, wsb)
    torch.cuda.synchronize()
    return [(E.cpu().numpy(), a.cpu().numpy(), b.cpu().numpy()) for E, a, b in zip(Es, dths, dxs)]


def _same(got, ref):
    for (E, dth, dx), (E1, dth1, dx1) in zip(got, ref):
        np.testing.assert_array_equal(E, E1)
        np.testing.assert_array_equal(dth, dth1)
        np.testing.assert_array_equal(dx, dx1)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("mode", MODES)
def test_batch_modes_equal_single_plans(mode):
    dev = torch.device("cuda:0")
    ws = mixed(10, (3, 14), (2, 8), 3, 31)
    circs, thetas, xs, dEs, xm, zm = _setup(ws, dev)
    ref = _single(circs, ws, thetas, xs, dEs, dev)
    batch = qfuse.Batch(circs, [w.x.shape[0] for w in ws], launch_mode=mode)
    wsb = batch.new_workspace(dev)
    got = _batch(batch, thetas, xs, dEs, wsb)
    _same(got, ref)
    # oracle
    orc = Oracle()
    for w, (E, dth, dx), d in zip(ws, got, dEs):
        Eo = orc.forward(w.n_qubits, w.gates, w.theta, w.x, xm, zm)
        _, dtho, dxo = orc.backward(w.n_qubits, w.gates, w.theta, w.x, xm, zm, d.cpu().numpy().astype(np.float64))
        assert np.abs(E - Eo).max() <= 1e-4
        assert np.abs(dth - dtho).max() <= 1e-3 * np.abs(dtho).max()
        assert np.abs(dx - dxo).max() <= 1e-3 * np.abs(dxo).max()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("mode", MODES)
def test_batch_uncompute_equals_single_plans(mode):
    """Uncompute mode in a mixed batch: the adjoint passes rebuild psi."""
    dev = torch.device("cuda:0")
    ws = mixed(8, (9, 15), (3, 8), 2, 33)
    circs, thetas, xs, dEs, xm, zm = _setup(ws, dev, seed=2)
    ref = _single(circs, ws, thetas, xs, dEs, dev, uncompute=1, ckpt_interval=2)
    batch = qfuse.Batch(circs, [w.x.shape[0] for w in ws], qfuse.make_tuning(uncompute=1, ckpt_interval=2),
                        launch_mode=mode)
    wsb = batch.new_workspace(dev)
    _same(_batch(batch, thetas, xs, dEs, wsb), ref)
    orc = Oracle()
    for w, (E, dth, dx), d in zip(ws, ref, dEs):
        _, dtho, dxo = orc.backward(w.n_qubits, w.gates, w.theta, w.x, xm, zm, d.cpu().numpy().astype(np.float64))
        assert np.abs(dth - dtho).max() <= 1e-3 * np.abs(dtho).max()
        assert np.abs(dx - dxo).max() <= 1e-3 * np.abs(dxo).max()


@pytest.mark.timeout(300)
def test_batch_graph_replays():
    """Replays with eager work and synchronisation between them, new values in the
    same buffers, then a new workspace address (graph captured again)."""
    dev = torch.device("cuda:0")
    ws = mixed(8, (10, 14), (3, 10), 4, 41)
    circs, thetas, xs, dEs, xm, zm = _setup(ws, dev, seed=1)
    batch = qfuse.Batch(circs, [4] * len(ws))
    wsb = batch.new_workspace(dev)
    rng = np.random.default_rng(7)
    for rep in range(4):
        if rep:
            for t in thetas:
                t.copy_(torch.tensor(rng.uniform(0, 6.283, size=t.numel()).astype(np.float32), device=dev))
            for d in dEs:
                d.mul_(-0.5)
        scratch = torch.randn(1 << 20, device=dev).sum()   # unrelated eager work between replays
        torch.cuda.synchronize()
        got = _batch(batch, thetas, xs, dEs, wsb)
        ref = _single(circs, ws, thetas, xs, dEs, dev)
        _same(got, ref)
        del scratch
    wsb2 = batch.new_workspace(dev)
    got = _batch(batch, thetas, xs, dEs, wsb2)
    _same(got, _single(circs, ws, thetas, xs, dEs, dev))


@pytest.mark.timeout(120)
def test_batch_errors():
    dev = torch.device("cuda:0")
    ws = mixed(3, (4, 6), (1, 2), 2, 51)
    circs, thetas, xs, dEs, xm, zm = _setup(ws, dev)
    batch = qfuse.Batch(circs, [2, 2, 2])
    with pytest.raises(qfuse.QFuseError):
        batch.set_launch_mode(7)
    small = torch.empty(256, dtype=torch.uint8, device=dev)
    with pytest.raises(qfuse.QFuseError):
        batch.forward(thetas, xs, small)
    with pytest.raises(qfuse.QFuseError):
        qfuse.Batch(circs, [2, 0, 2])
    with pytest.raises(qfuse.QFuseError):
        qfuse.Batch(circs, [2, 2, 2], qfuse.make_tuning(mode=1))
    info = batch.info
    assert info.n_circuits == 3 and info.samples == 6
    assert info.fwd_launches <= info.fwd_jobs
