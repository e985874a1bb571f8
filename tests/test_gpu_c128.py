"""The complex128 validation path (tuning mode 2) through the C-ABI.

It computes the same expectations and adjoint gradients as the oracle in double
precision, one kernel per gate, so the two agree to rounding: |dE| <= 1e-10 and
normwise relative gradient error <= 1e-9.  Its autograd wrapper passes
torch.autograd.gradcheck (central finite differences in double precision).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import CZ, RX, RY, RZ, hea_gates, z_observables  # noqa: E402

pytestmark = pytest.mark.gpu

E_TOL = 1e-10
G_TOL = 1e-9
C128 = qfuse.make_tuning(mode=qfuse.QF_MODE_C128)


def rel(a, b):
    s = float(np.abs(b).max()) if np.size(b) else 0.0
    d = float(np.abs(np.asarray(a) - b).max()) if np.size(b) else 0.0
    return d / s if s > 0 else d


def run_c128(n, gates, theta, x, zm, dE, micro_batch=0):
    dev = torch.device("cuda:0")
    circ = qfuse.Circuit(n, gates, len(theta), x.shape[1], zm)
    plan = qfuse.Plan(circ, x.shape[0], qfuse.make_tuning(mode=qfuse.QF_MODE_C128, micro_batch=micro_batch))
    ws = plan.new_workspace(dev)
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    xx = torch.tensor(x, dtype=torch.float64, device=dev) if x.shape[1] else None
    E = plan.forward(th, xx, ws)
    dth, dx = plan.backward(th, xx, torch.tensor(dE, dtype=torch.float64, device=dev), ws)
    torch.cuda.synchronize()
    return E.cpu().numpy(), dth.cpu().numpy(), (dx.cpu().numpy() if dx is not None else np.zeros_like(x))


@pytest.mark.parametrize("n,L,rots,B,obs,mb", [
    (1, 2, ("RX", "RY", "RZ"), 2, [0], 0),
    (4, 3, ("RY", "RZ"), 3, [0, 2], 0),
    (6, 4, ("RX", "RY", "RZ"), 5, [0, 1, 5], 2),     # several micro-batches, ragged tail
    (9, 2, ("RX", "RY", "RZ"), 2, list(range(9)), 0),
    (12, 2, ("RY", "RZ"), 2, [0, 11], 0),            # more than one partial-sum block per gate
])
def test_c128_matches_oracle(n, L, rots, B, obs, mb):
    rng = np.random.default_rng(1000 + n)
    gates = hea_gates(n, L, rots)
    P = L * len(rots) * n
    theta = rng.uniform(-np.pi, np.pi, P)
    x = rng.uniform(-np.pi, np.pi, (B, n))
    xm, zm = z_observables(obs)
    dE = rng.normal(size=(B, len(obs)))
    E, dth, dx = run_c128(n, gates, theta, x, zm, dE, micro_batch=mb)
    Eo, dtho, dxo = Oracle().backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL, np.abs(E - Eo).max()
    assert rel(dth, dtho) <= G_TOL, rel(dth, dtho)
    assert rel(dx, dxo) <= G_TOL, rel(dx, dxo)


def test_c128_general_gate_list_with_shared_angles():
    # runs of mixed kinds on one qubit, CZ between distant qubits, angles shared
    # by several gates, and an input angle used twice
    n = 5
    gates = np.array([
        [RX, 0, -1, 0, -1], [RY, 0, -1, 1, -1], [RZ, 0, -1, 0, -1],
        [RY, 3, -1, -1, 1], [CZ, 0, 4, -1, -1], [RZ, 4, -1, 2, -1],
        [RX, 2, -1, -1, 1], [CZ, 3, 1, -1, -1], [RY, 1, -1, 2, -1], [RX, 3, -1, 1, -1],
    ], dtype=np.int32)
    rng = np.random.default_rng(7)
    theta = rng.uniform(-3, 3, 3)
    x = rng.uniform(-3, 3, (3, 2))
    xm, zm = z_observables([0, 3])
    dE = rng.normal(size=(3, 2))
    E, dth, dx = run_c128(n, gates, theta, x, zm, dE)
    Eo, dtho, dxo = Oracle().backward(n, gates, theta, x, xm, zm, dE)
    assert np.abs(E - Eo).max() <= E_TOL
    assert rel(dth, dtho) <= G_TOL and rel(dx, dxo) <= G_TOL


def test_c128_gradcheck():
    dev = torch.device("cuda:0")
    n, L = 3, 2
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    P = L * 3 * n
    xm, zm = z_observables([0, 2])
    circ = qfuse.Circuit(n, gates, P, n, zm)
    plan = qfuse.Plan(circ, 2, C128)
    g = torch.Generator().manual_seed(3)
    theta = (torch.rand(P, generator=g, dtype=torch.float64) * 6 - 3).to(dev).requires_grad_()
    x = (torch.rand(2, n, generator=g, dtype=torch.float64) * 6 - 3).to(dev).requires_grad_()
    assert torch.autograd.gradcheck(lambda t, xx: qfuse.circuit_expectations(t, xx, plan, True), (theta, x),
                                    eps=1e-6, atol=1e-7, rtol=1e-5)


def test_c128_and_float_paths_reject_each_other():
    dev = torch.device("cuda:0")
    gates = hea_gates(3, 1, ("RY",))
    xm, zm = z_observables([0])
    circ = qfuse.Circuit(3, gates, 3, 3, zm)
    p64 = qfuse.Plan(circ, 1, C128)
    p32 = qfuse.Plan(circ, 1)
    ws = torch.empty(max(p64.ws_bytes, p32.ws_bytes), dtype=torch.uint8, device=dev)
    th32, x32 = torch.zeros(3, device=dev), torch.zeros(1, 3, device=dev)
    E32 = torch.empty(1, 1, device=dev)
    th64, x64, E64 = th32.double(), x32.double(), E32.double()
    s = None
    with pytest.raises(qfuse.QFuseError) as e:
        qfuse.qf_forward(p64.handle, th32, x32, E32, ws, ws.numel(), s)
    assert e.value.status == 1
    with pytest.raises(qfuse.QFuseError) as e:
        qfuse.qf_forward_c128(p32.handle, th64, x64, None, E64, ws, ws.numel(), s)
    assert e.value.status == 1
    with pytest.raises(ValueError):
        p64.forward(th32, x32, ws)


def test_float_per_gate_close_to_c128():
    n, L, B = 8, 3, 3
    rng = np.random.default_rng(11)
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    theta = rng.uniform(-np.pi, np.pi, L * 3 * n)
    x = rng.uniform(-np.pi, np.pi, (B, n))
    xm, zm = z_observables([0, 4])
    dE = rng.normal(size=(B, 2))
    E64, dth64, dx64 = run_c128(n, gates, theta, x, zm, dE)
    dev = torch.device("cuda:0")
    circ = qfuse.Circuit(n, gates, len(theta), n, zm)
    plan = qfuse.Plan(circ, B, qfuse.make_tuning(mode=qfuse.QF_MODE_PER_GATE))
    ws = plan.new_workspace(dev)
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    xx = torch.tensor(x, dtype=torch.float32, device=dev)
    E = plan.forward(th, xx, ws)
    dth, dx = plan.backward(th, xx, torch.tensor(dE, dtype=torch.float32, device=dev), ws)
    # float32 inputs are the rounded doubles: compare at the float path's tolerance
    assert np.abs(E.cpu().numpy() - E64).max() <= 1e-4
    assert rel(dth.cpu().numpy(), dth64) <= 1e-3 and rel(dx.cpu().numpy(), dx64) <= 1e-3
