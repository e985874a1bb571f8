"""Randomised plans and mixed batches on the GPU against the oracle: the seeded random
circuits and execution choices of the CPU randomised tests (1-9 qubits, RX/RY/RZ subsets,
CZ or CNOT ladders or rings; random tile and register qubits, fusion depth, end-of-pass
epoch threshold, uncompute mode, checkpoint interval and micro-batch), run through the HIP
kernels (paper Sec. 2.1 expectation, Sec. 2.2 adjoint gradient)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import z_observables  # noqa: E402
from random_cases import close, random_batch_tuning, random_circuit, random_tuning, random_tuning_wide  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return Oracle()


@pytest.mark.timeout(120)
@pytest.mark.parametrize("seed", range(200))
def test_random_plan_gpu(orc, seed):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(1000 + seed)
    n, gates, theta, x, obs = random_circuit(rng, seed)
    tun = random_tuning(rng, n, x.shape[0])
    xm, zm = z_observables(obs)
    dE = rng.normal(size=(x.shape[0], len(obs))).astype(np.float32)
    print(f"seed {seed}: n={n} batch={x.shape[0]} tuning={tun}", flush=True)
    circ = qfuse.Circuit(n, gates, len(theta), n, zm)
    plan = qfuse.Plan(circ, x.shape[0], qfuse.make_tuning(**tun))
    ws = plan.new_workspace(dev)
    th = torch.tensor(theta, device=dev)
    xx = torch.tensor(x, device=dev)
    E = plan.forward(th, xx, ws)
    dth, dx = plan.backward(th, xx, torch.tensor(dE, device=dev), ws)
    torch.cuda.synchronize()
    got = (E.cpu().numpy(), dth.cpu().numpy(), dx.cpu().numpy())
    assert close(*got, orc.backward(n, gates, theta, x, xm, zm, dE)), (n, tun)


@pytest.mark.timeout(120)
@pytest.mark.parametrize("seed", range(30))
def test_random_wide_plan_gpu(orc, seed):
    """10..16 qubits: several tiles, swaps to local, random supported tile shapes."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(9000 + seed)
    n = 0
    while n < 10:
        n, gates, theta, x, obs = random_circuit(rng, seed, max_n=16)
    tun = random_tuning_wide(rng, n, x.shape[0])
    xm, zm = z_observables(obs)
    dE = rng.normal(size=(x.shape[0], len(obs))).astype(np.float32)
    print(f"seed {seed}: n={n} batch={x.shape[0]} tuning={tun}", flush=True)
    circ = qfuse.Circuit(n, gates, len(theta), n, zm)
    plan = qfuse.Plan(circ, x.shape[0], qfuse.make_tuning(**tun))
    ws = plan.new_workspace(dev)
    th = torch.tensor(theta, device=dev)
    xx = torch.tensor(x, device=dev)
    E = plan.forward(th, xx, ws)
    dth, dx = plan.backward(th, xx, torch.tensor(dE, device=dev), ws)
    torch.cuda.synchronize()
    got = (E.cpu().numpy(), dth.cpu().numpy(), dx.cpu().numpy())
    assert close(*got, orc.backward(n, gates, theta, x, xm, zm, dE)), (n, tun)


@pytest.mark.timeout(120)
@pytest.mark.parametrize("seed", range(40))
def test_random_batch_gpu(orc, seed):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5000 + seed)
    circs, samples, thetas, xs, dEs, refs = [], [], [], [], [], []
    for i in range(int(rng.integers(1, 7))):
        n, gates, theta, x, obs = random_circuit(rng, 10 * seed + i)
        xm, zm = z_observables(obs)
        dE = rng.normal(size=(x.shape[0], len(obs))).astype(np.float32)
        circs.append(qfuse.Circuit(n, gates, len(theta), n, zm))
        samples.append(x.shape[0])
        thetas.append(torch.tensor(theta, device=dev))
        xs.append(torch.tensor(x, device=dev))
        dEs.append(torch.tensor(dE, device=dev))
        refs.append(orc.backward(n, gates, theta, x, xm, zm, dE))
    tun = random_batch_tuning(rng)
    print(f"seed {seed}: {len(circs)} circuits, tuning={tun}", flush=True)
    batch = qfuse.Batch(circs, samples, qfuse.make_tuning(**tun))
    ws = batch.new_workspace(dev)
    Es = batch.forward(thetas, xs, ws)
    dths, dxs = batch.backward(thetas, xs, dEs, ws)
    torch.cuda.synchronize()
    for i, ref in enumerate(refs):
        assert close(Es[i].cpu().numpy(), dths[i].cpu().numpy(), dxs[i].cpu().numpy(), ref), (i, tun)
