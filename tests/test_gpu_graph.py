"""A plan's forward and backward captured into a HIP graph (through torch's
graph capture on the current stream) and replayed: every replay gives the
eager results bit for bit, with eager work and new inputs between replays.
The calls launch kernels only (no allocation, no memset), so they capture."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_02804_amd import qfuse  # noqa: E402
from paper_2603_02804_amd.workloads import draw_inputs, hea_gates, z_observables  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,L,tun", [(14, 6, dict(ckpt_interval=2, micro_batch=2)), (9, 4, {}),
                                     (13, 5, dict(mem_save=1, ckpt_interval=2)),
                                     (14, 5, dict(uncompute=1, ckpt_interval=2))])
def test_plan_graph_replays(n, L, tun):
    dev = torch.device("cuda:0")
    B = 4
    gates = hea_gates(n, L, ("RX", "RY", "RZ"))
    theta_np, x_np, _ = draw_inputs(150 + n, L * 3 * n, B, n)
    xm, zm = z_observables([0, n - 1])
    circ = qfuse.Circuit(n, gates, len(theta_np), n, zm)
    plan = qfuse.Plan(circ, B, qfuse.make_tuning(**tun) if tun else None)
    ws = plan.new_workspace(dev)
    theta = torch.tensor(theta_np, device=dev)
    x = torch.tensor(x_np, device=dev)
    dE = torch.tensor(np.random.default_rng(n).normal(size=(B, 2)).astype(np.float32), device=dev)
    E = torch.empty(B, 2, device=dev)
    dth = torch.empty_like(theta)
    dx = torch.empty_like(x)
    s = lambda: torch.cuda.current_stream().cuda_stream  # noqa: E731

    def run():
        qfuse.qf_forward(plan.handle, theta, x, E, ws, ws.numel(), s())
        qfuse.qf_backward(plan.handle, theta, x, dE, dth, dx, ws, ws.numel(), s())

    run()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (E, dth, dx)]
    # warm up on a side stream, then capture
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for rep in range(3):
        E.zero_(); dth.zero_(); dx.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((E, dth, dx), ref):
            assert torch.equal(a, b), f"replay {rep}"
        _ = (theta * 2).sum().item()     # eager work between replays
    # new inputs in the same buffers: the graph follows them
    theta.mul_(0.5)
    g.replay()
    torch.cuda.synchronize()
    got = [t.clone() for t in (E, dth, dx)]
    run()
    torch.cuda.synchronize()
    for a, b in zip(got, (E, dth, dx)):
        assert torch.equal(a, b)
