"""Benchmark: samples/s of forward + adjoint gradient on a 20-qubit, 1000-layer HEA.

One step = forward to the expectations <Z_0..Z_9> of a batch of 1000 samples,
10-class softmax cross-entropy in torch, and the fused adjoint backward to
dL/dtheta (60000 angles, summed over the batch) and dL/dx (20 encoding angles
per sample).  Inputs are resident in HBM before the timed region.

Printed (one JSON line): throughput, the roofline position of the dominant
kernel (the fused adjoint pass, timed live with HIP events around its launches),
the unfused one-kernel-per-gate path on the same GPU, and the complex128 CPU
oracle on the host cores (bounded sample, extrapolated).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "samples/s fwd+adjoint grad (20q×1000L HEA) fused vs per-gate; HBM GB/s % peak"
PEAK_HBM_GBS = 8000.0
# MI355X FP32 vector peak as published: 256 CUs x 128 FP32 FMA lanes per clock
# (packed FP32) x 2 flops x 2.4 GHz = 157.3 TFLOP/s.  This build disables packed
# FP32 instructions, which halves the attainable rate (78.6 TFLOP/s); both are
# reported.
PEAK_FP32_TFLOPS = 256 * 128 * 2 * 2.4e9 / 1e12
PEAK_FP32_UNPACKED_TFLOPS = PEAK_FP32_TFLOPS / 2
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bwd_pass_hea20q1000l.json")
# sources that decide what the pass kernels execute and read/write: when any of
# them changes, the stored counter measurement no longer applies
KERNEL_SRCS = [os.path.join(ROOT, "paper_2603_02804_amd", "csrc", f)
               for f in ("device.hpp", "kargs.hpp", "plan_types.hpp", "plan.cpp")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="hea20q1000l",
                    choices=("hea20q1000l", "hea16q200l", "hea12q100l", "mixed256", "paper20q1000l", "hea_d1_sweep"),
                    help="hea20q1000l: the headline 20-qubit, 1000-layer HEA (batch 1000); hea16q200l: 16 qubits, "
                         "200 layers, batch 512; hea12q100l: 12 qubits, 100 layers, batch 1024; mixed256: 256 mixed "
                         "circuits, one merged HIP graph vs per-circuit launches; paper20q1000l: the paper's Table 1 "
                         "shape; hea_d1_sweep: one-layer HEA from random states, 4..20 qubits, fused vs per-gate")
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=0, help="override the batch (exploration only)")
    ap.add_argument("--layers", type=int, default=0, help="override the depth (exploration only)")
    ap.add_argument("--fusion-depth", type=int, default=0)
    ap.add_argument("--ckpt-interval", type=int, default=0)
    ap.add_argument("--micro-batch", type=int, default=0)
    ap.add_argument("--tile-qubits", type=int, default=0)
    ap.add_argument("--reg-qubits", type=int, default=0)
    ap.add_argument("--uncompute", type=int, choices=(0, 1), default=None,
                    help="1: adjoint passes rebuild psi (no recompute); 0: recompute segments (default: autotuned, "
                         "else 1)")
    ap.add_argument("--epoch-fill", type=int, default=0,
                    help="end-of-pass epochs with fewer runs wait for the next pass (0: register qubits, -1: none)")
    ap.add_argument("--no-baselines", action="store_true", help="skip the per-gate and CPU baselines")
    ap.add_argument("--no-autotune", action="store_true", help="ignore the cached autotuned configuration")
    ap.add_argument("--pg-samples", type=int, default=8)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    return ap.parse_args()


def kernel_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(samples are independent, so a multi-GPU run would shard the batch and all-reduce dL/dtheta)",
              file=sys.stderr)
        return 2
    import torch

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}), flush=True)
        return 0

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "mixed256":
        return bench_mixed(args, dev)
    if args.workload == "paper20q1000l":
        return bench_paper(args, dev)
    if args.workload == "hea_d1_sweep":
        return bench_sweep(args, dev)
    return bench_hea(args, dev)


def host_info() -> dict:
    """The host the CPU baseline ran on: usable cores and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"nproc": nproc, "cpu_model": model}


def hea_workload(name, layers=0):
    from paper_2603_02804_amd.workloads import c2, c3, c4, make_workload
    if name == "hea20q1000l" and layers:
        return make_workload("hea20q", 20, layers, ("RX", "RY", "RZ"), 1000, tuple(range(10)), "ce", 4)
    return {"hea12q100l": c2, "hea16q200l": c3, "hea20q1000l": c4}[name]()


def metric_of(w) -> str:
    if w.name == "hea20q1000l" and w.n_layers == 1000:
        return METRIC
    rots = "".join(r[1] for r in w.rotations)
    return (f"samples/s fwd+adjoint grad ({w.n_qubits}q×{w.n_layers}L HEA, R{rots} + CZ ladder) fused vs per-gate; "
            "HBM GB/s % peak")


def describe(w) -> str:
    rots = ",".join(w.rotations)
    loss = (f"<Z_0..Z_{w.n_obs - 1}> -> {w.n_obs}-class CE" if w.loss == "ce"
            else f"mean of <Z_i> over {w.n_obs} qubits, summed over the batch")
    return (f"{w.name}: {w.n_qubits}-qubit HEA, {w.n_layers} layers of {rots} + CZ ladder, {w.n_params} angles, "
            f"RY encoding of {w.n_inputs} features, {loss}")


def bench_hea(args, dev) -> int:
    """One of the HEA configurations: fused forward, loss in torch, fused adjoint backward."""
    import numpy as np
    import torch
    import torch.nn.functional as Fnn

    from paper_2603_02804_amd import qfuse

    w = hea_workload(args.workload, args.layers)
    B = args.batch or w.batch
    x_np = w.x[:B]
    lab_np = w.labels[:B]

    unc = 1 if args.uncompute is None else args.uncompute
    tun = qfuse.make_tuning(fusion_depth=args.fusion_depth, ckpt_interval=args.ckpt_interval,
                            micro_batch=args.micro_batch, tile_qubits=args.tile_qubits,
                            reg_qubits=args.reg_qubits, epoch_fill=args.epoch_fill, uncompute=unc)
    tuning_src = "flags" if any((args.fusion_depth, args.ckpt_interval, args.micro_batch, args.tile_qubits,
                                 args.reg_qubits, args.epoch_fill, args.uncompute is not None)) else "default"
    if tuning_src == "default" and not args.no_autotune:
        from paper_2603_02804_amd import autotune
        cached = autotune.cached_tuning(w.n_qubits, w.gates, w.n_obs, B, autotune.device_key(dev))
        if cached:
            tun = autotune.tuning_from(cached)
            tuning_src = "autotuned (paper_2603_02804_amd/tuned_configs.json)"
    circ = qfuse.Circuit(w.n_qubits, w.gates, w.n_params, w.n_inputs, w.zmask)
    plan = qfuse.Plan(circ, B, tun)
    info = plan.info
    theta = torch.tensor(w.theta, device=dev, requires_grad=True)
    x = torch.tensor(x_np, device=dev, requires_grad=True)
    labels = torch.tensor(lab_np, device=dev)

    def loss_of(E, lab):
        if w.loss == "ce":
            return Fnn.cross_entropy(E, lab)
        return E.mean(dim=1).sum()

    def step():
        theta.grad = None
        x.grad = None
        E = qfuse.circuit_expectations(theta, x, plan)
        loss = loss_of(E, labels)
        loss.backward()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    qfuse.qf_profile_enable(plan.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = qfuse.qf_profile_read(plan.handle)
    qfuse.qf_profile_enable(plan.handle, False)
    elapsed = t1 - t0
    value = B * args.steps / elapsed
    ms_step = 1000.0 * elapsed / args.steps

    # dominant kernel: the fused adjoint pass
    n_bwd = int(prof.launches[1])
    bwd_s = prof.ms[1] / 1000.0
    n_fwd = int(prof.launches[0])
    fwd_s = prof.ms[0] / 1000.0
    flops_bwd = info.bwd_pass_flops_per_sample * B * args.steps
    bytes_bwd = info.bwd_pass_bytes_per_sample * B * args.steps
    achieved_tf = flops_bwd / bwd_s / 1e12 if bwd_s > 0 else 0.0
    traffic = None
    if os.path.exists(TRAFFIC_FILE) and w.name == "hea20q1000l":
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        # per-sample bytes depend on the pass structure, not on how samples are grouped into micro-batches
        shape = {k: getattr(info, k) for k in ("tile_qubits", "reg_qubits", "fusion_depth", "fused_passes",
                                               "uncompute")}
        if tr.get("kernel_src_sha") == kernel_sha() and tr.get("plan") == shape and not args.layers:
            # counters were taken per sample over every adjoint pass launch
            traffic = round(tr["hbm_bytes_per_sample"] * B * args.steps / max(1, n_bwd))
    roofline = {
        "kernel": f"k_pass<{info.reg_qubits},{info.threads},true> (fused adjoint pass)",
        "bound": "alu", "achieved": round(achieved_tf, 2), "peak": round(PEAK_FP32_TFLOPS, 1), "unit": "TFLOP/s",
        "frac": round(achieved_tf / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
        "peak_unpacked": round(PEAK_FP32_UNPACKED_TFLOPS, 1),
        "executed_tflops": round(info.exec_bwd_pass_flops_per_sample * B * args.steps / bwd_s / 1e12, 2)
        if bwd_s > 0 else 0.0,
        "flops_per_run_amplitude": 48,
        "launches": n_bwd, "avg_launch_ms": round(prof.ms[1] / max(1, n_bwd), 4),
        "flops_per_launch": flops_bwd / max(1, n_bwd), "bytes_per_launch": bytes_bwd / max(1, n_bwd),
        "hbm_gbs": round(bytes_bwd / bwd_s / 1e9, 1) if bwd_s > 0 else 0.0,
    }
    # the forward pass kernel beside it (16 algorithmic flops per run-amplitude, 6 executed)
    fwd_flops = info.fwd_flops_per_sample * B * args.steps
    fwd_tf = fwd_flops / fwd_s / 1e12 if fwd_s > 0 else 0.0
    fwd_roof = {"kernel": f"k_pass<{info.reg_qubits},{info.threads},false> (fused forward pass)",
                "achieved": round(fwd_tf, 2), "frac": round(fwd_tf / PEAK_FP32_TFLOPS, 4),
                "executed_tflops": round(fwd_tf * 6 / 16, 2), "launches": n_fwd,
                "avg_launch_ms": round(prof.ms[0] / max(1, n_fwd), 4),
                "hbm_gbs": round(info.fwd_bytes_per_sample * B * args.steps / fwd_s / 1e9, 1) if fwd_s > 0 else 0.0}
    step_bytes = (info.fwd_bytes_per_sample + info.bwd_bytes_per_sample) * B
    hbm_gbs = step_bytes / (elapsed / args.steps) / 1e9
    kernel_share = {"fwd_pass_ms": round(prof.ms[0] / args.steps, 1), "bwd_pass_ms": round(prof.ms[1] / args.steps, 1),
                    "other_ms": round(prof.ms[2] / args.steps, 1)}
    out = {
        "metric": metric_of(w), "value": round(value, 3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": describe(w) if not args.layers else f"{w.name}{w.n_layers}l (depth override)",
                   "batch": B, "micro_batch": info.micro_batch, "tile_qubits": info.tile_qubits,
                   "reg_qubits": info.reg_qubits, "fusion_depth": info.fusion_depth, "fused_passes": info.fused_passes,
                   "ckpt_interval": info.ckpt_interval, "segments": info.segments, "epoch_fill": info.epoch_fill,
                   "uncompute": info.uncompute, "tuning": tuning_src},
        "roofline": roofline,
        "forward_pass": fwd_roof,
        "hbm": {"gbs": round(hbm_gbs, 1), "frac": round(hbm_gbs / PEAK_HBM_GBS, 4),
                "bytes_per_sample": info.fwd_bytes_per_sample + info.bwd_bytes_per_sample},
        "kernel_time_per_step": kernel_share,
        "loss": float(loss.detach().cpu()),
    }

    if not args.no_baselines:
        # unfused one-kernel-per-gate path on the same GPU (same circuit, full depth)
        nb = min(args.pg_samples, B)
        pg_plan = qfuse.Plan(circ, nb, qfuse.make_tuning(mode=1, micro_batch=nb))
        th2 = theta.detach()
        x2 = x.detach()[:nb].contiguous()
        ws = pg_plan.new_workspace(dev)
        lab2 = labels[:nb]

        def pg_step():
            E = pg_plan.forward(th2, x2, ws)
            Ev = E.clone().requires_grad_(True)
            loss_of(Ev, lab2).backward()
            pg_plan.backward(th2, x2, Ev.grad, ws)

        pg_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pg_step()
        torch.cuda.synchronize()
        pg_s = time.perf_counter() - t0
        pg_value = nb / pg_s
        pgi = pg_plan.info
        pg_gbs = (pgi.fwd_bytes_per_sample + pgi.bwd_bytes_per_sample) * pg_value / 1e9
        out["per_gate"] = {"value": round(pg_value, 3), "unit": "samples/s", "sample": f"{nb} samples, full depth",
                           "speedup_fused": round(value / pg_value, 2),
                           # the unfused kernels are HBM-bound: their algorithmic bytes over time
                           "hbm_gbs": round(pg_gbs, 1), "hbm_frac": round(pg_gbs / PEAK_HBM_GBS, 4)}
        del ws
        out["cpu_baseline"] = cpu_baseline_hea(w, x_np, lab_np, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


def cpu_baseline_hea(w, x_np, lab_np, budget_s):
    """The complex128 oracle on the host cores: forward + adjoint gradient of a bounded sample of the
    workload.  Full depth for as many samples as fit the time budget; a circuit too deep for one
    sample in the budget is timed on its leading layers and extrapolated linearly in depth."""
    import numpy as np

    from oracle.oracle import Oracle, loss_and_grad_E
    from paper_2603_02804_amd.workloads import hea_gates
    orc = Oracle()
    n, R = w.n_qubits, len(w.rotations)

    def cpu_time(L, nb):
        g = hea_gates(n, L, w.rotations)
        _, gE = loss_and_grad_E(np.zeros((nb, w.n_obs)), w.loss, lab_np[:nb])
        t = time.perf_counter()
        orc.backward(n, g, w.theta[:L * R * n], x_np[:nb], w.xmask, w.zmask, gE)
        return time.perf_counter() - t

    t1l = cpu_time(1, 1)
    if t1l * w.n_layers <= budget_s / 2:
        t_full = cpu_time(w.n_layers, 1)
        nb = int(max(1, min(len(x_np), budget_s // max(t_full, 1e-6))))
        t = cpu_time(w.n_layers, nb) if nb > 1 else t_full
        per_sample = t / nb
        sample = f"{nb} samples at full depth ({t:.1f} s)"
    else:
        Ls = int(max(1, min(w.n_layers, round(budget_s / max(t1l, 1e-3)))))
        tL = cpu_time(Ls, 1) if Ls > 1 else t1l
        per_sample = tL * w.n_layers / Ls
        sample = f"1 sample, first {Ls} of {w.n_layers} layers ({tL:.1f} s), extrapolated linearly in depth"
    return {"value": round(1.0 / per_sample, 6), "unit": "samples/s", "cores": orc.num_threads, "kind": "oracle",
            "sample": sample, "host": host_info()}


# The paper's own 20-qubit, 1000-layer epoch (Table 1, fused, GH200): 1,000 samples in 1,273 s.
PAPER_EPOCH_SAMPLES_PER_S = 1000 / 1273.0


def bench_paper(args, dev) -> int:
    """The paper's experiment shape (Sec. 4, Table 1): 20 qubits, 1000 layers of RX, RY, RZ closed by a
    CZ ring, random initial states, O = (IXYZ)^5, L = sum of E, batch 1000."""
    import numpy as np
    import torch

    from paper_2603_02804_amd import autotune, qfuse
    from paper_2603_02804_amd.workloads import hea_gates, pauli_string

    n, L = 20, args.layers or 1000
    B = args.batch or 1000
    gates = hea_gates(n, L, ("RX", "RY", "RZ"), encoding=False, ring=True)
    rng = np.random.default_rng(6)
    theta = torch.tensor(rng.uniform(0.0, 2.0 * np.pi, L * 3 * n).astype(np.float32), device=dev)
    # random states: independent standard normal parts from a seeded generator on the device, unit norm
    g = torch.Generator(device=dev).manual_seed(6)
    psi0 = torch.complex(torch.randn(B, 1 << n, generator=g, device=dev),
                         torch.randn(B, 1 << n, generator=g, device=dev))
    psi0 /= torch.linalg.vector_norm(psi0, dim=1, keepdim=True)
    xm, zm = pauli_string(("IXYZ" * 5)[:n])
    circ = qfuse.Circuit(n, gates, L * 3 * n, 0, [zm], [xm])
    unc = 1 if args.uncompute is None else args.uncompute
    tun = qfuse.make_tuning(micro_batch=args.micro_batch or 512, fusion_depth=args.fusion_depth,
                            ckpt_interval=args.ckpt_interval, tile_qubits=args.tile_qubits,
                            reg_qubits=args.reg_qubits, epoch_fill=args.epoch_fill, uncompute=unc)
    probe = qfuse.Plan(circ, B, tun)
    if not args.ckpt_interval:
        mb = probe.info.micro_batch
        if unc:
            store, c = autotune.uncompute_storage(probe.info.fused_passes, B, mb, 8 << n,
                                                  0.85 * torch.cuda.mem_get_info()[0])
        else:
            store, c = 1, autotune.optimal_ckpt(probe.info.fused_passes, B, mb, True)
        tun = qfuse.make_tuning(micro_batch=mb, fusion_depth=args.fusion_depth, ckpt_interval=c,
                                tile_qubits=args.tile_qubits, reg_qubits=args.reg_qubits,
                                epoch_fill=args.epoch_fill, uncompute=unc, store_ckpt=store)
    del probe
    plan = qfuse.Plan(circ, B, tun)
    info = plan.info
    theta.requires_grad_(True)

    def step():
        theta.grad = None
        E = qfuse.circuit_expectations(theta, None, plan, psi0=psi0)
        E.sum().backward()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    value = B / sec
    out = {
        "metric": "samples/s fwd+adjoint grad, the paper's 20-qubit 1000-layer epoch shape",
        "value": round(value, 3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000 * sec, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": round(value / PAPER_EPOCH_SAMPLES_PER_S, 2) if (L == 1000 and B == 1000) else None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"paper20q{L}l: 20-qubit HEA, {L} layers of RX,RY,RZ + CZ ring, random initial "
                               "states, O = (IXYZ)^5, L = sum E",
                   "batch": B, "micro_batch": info.micro_batch, "fused_passes": info.fused_passes,
                   "ckpt_interval": info.ckpt_interval, "segments": info.segments, "uncompute": info.uncompute,
                   "paper": "1,273 s per 1,000-sample epoch on GH200 (Table 1): 0.786 samples/s; context, "
                            "other hardware"},
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_sweep(args, dev) -> int:
    """The paper's throughput experiment (Sec. 4.2): a one-layer HEA (RX, RY, RZ on every qubit, CZ ring)
    applied to random initial states, observable (IXYZ) repeated over the register, L = sum of E;
    forward + adjoint gradient, fused and per gate, for 4..20 qubits.  The batch per size is the largest
    power of two up to 65536 whose states take at most 4 GiB (the paper takes the largest batch that fits
    its GPU)."""
    import numpy as np
    import torch

    from paper_2603_02804_amd import qfuse
    from paper_2603_02804_amd.workloads import paper_mode

    sizes = list(range(4, 21)) if not args.layers else [args.layers]
    rows = []
    for n in sizes:
        B = args.batch or int(min(65536, max(64, (4 << 30) // (8 << n))))
        w = paper_mode(n, 1, 1, seed=n)
        g = torch.Generator(device=dev).manual_seed(n)
        psi0 = torch.complex(torch.randn(B, 1 << n, generator=g, device=dev),
                             torch.randn(B, 1 << n, generator=g, device=dev))
        psi0 /= torch.linalg.vector_norm(psi0, dim=1, keepdim=True)
        theta = torch.tensor(w.theta, device=dev)
        circ = qfuse.Circuit(n, w.gates, len(w.theta), 0, w.zmask, w.xmask)
        dE = torch.ones(B, 1, device=dev)

        def timed(plan, nb, reps):
            ws = plan.new_workspace(dev)
            p0 = psi0[:nb]
            d = dE[:nb]

            def once():
                plan.forward(theta, None, ws, psi0=p0)
                plan.backward(theta, None, d, ws, psi0=p0)

            once()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                once()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t) / reps
            del ws
            return sec

        # the whole batch in one micro-batch: a one-layer circuit has two passes, each a short launch
        plan = qfuse.Plan(circ, B, qfuse.make_tuning(uncompute=1, micro_batch=B))
        info = plan.info
        sec = timed(plan, B, max(1, args.steps))
        # algorithmic bytes of the call: the plan's passes plus the initial-state read
        byts = (info.fwd_bytes_per_sample + info.bwd_bytes_per_sample + (8 << n)) * B
        nb_pg = min(B, 4096)
        pg = qfuse.Plan(circ, nb_pg, qfuse.make_tuning(mode=1, micro_batch=nb_pg))
        pg_sec = timed(pg, nb_pg, 1)
        pgi = pg.info
        pg_bytes = (pgi.fwd_bytes_per_sample + pgi.bwd_bytes_per_sample + (8 << n)) * nb_pg
        del plan, pg
        row = {"n": n, "batch": B, "fused_passes": info.fused_passes, "fused": round(B / sec, 1),
               "per_gate": round(nb_pg / pg_sec, 1), "speedup": round((B / sec) / (nb_pg / pg_sec), 2),
               "fused_hbm_gbs": round(byts / sec / 1e9, 1), "fused_hbm_frac": round(byts / sec / 1e9 / PEAK_HBM_GBS, 4),
               "per_gate_hbm_gbs": round(pg_bytes / pg_sec / 1e9, 1)}
        rows.append(row)
        print(json.dumps({"sweep_row": row}), file=sys.stderr, flush=True)
        del psi0
        torch.cuda.empty_cache()
    last = rows[-1]
    out = {
        "metric": "samples/s fwd+adjoint grad, one-layer HEA (RX,RY,RZ + CZ ring) from random states, fused vs "
                  "per-gate, 4..20 qubits",
        "value": last["fused"], "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(1000 * last["batch"] / last["fused"], 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"hea_d1_sweep: one layer of RX,RY,RZ + CZ ring, random initial states, O = (IXYZ)... "
                               f"over the register, L = sum E; value at {last['n']} qubits, batch {last['batch']}",
                   "uncompute": 1},
        "sweep": rows,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_mixed(args, dev) -> int:
    """256 circuits, qubits ~ U{10..18}, layers ~ U{50..500} (RY,RZ + CZ ladder), 4 samples each,
    L = sum of <Z_0>: forward + adjoint gradient of every circuit in one step."""
    import numpy as np
    import torch

    from paper_2603_02804_amd import qfuse
    from paper_2603_02804_amd.workloads import c5, z_observables

    ws = c5()
    xm, zm = z_observables([0])
    circs = [qfuse.Circuit(c.n_qubits, c.gates, len(c.theta), c.n_qubits, zm) for c in ws]
    samples = [c.x.shape[0] for c in ws]
    thetas = [torch.tensor(c.theta, device=dev) for c in ws]
    xs = [torch.tensor(c.x, device=dev) for c in ws]
    dEs = [torch.ones(s, 1, device=dev) for s in samples]
    t0 = time.perf_counter()
    unc = 1 if args.uncompute is None else args.uncompute
    batch = qfuse.Batch(circs, samples, qfuse.make_tuning(epoch_fill=args.epoch_fill, uncompute=unc,
                                                           fusion_depth=args.fusion_depth))
    t_create = time.perf_counter() - t0
    info = batch.info
    wsb = batch.new_workspace(dev)
    n_samples = int(info.samples)

    def step():
        batch.forward(thetas, xs, wsb)
        batch.backward(thetas, xs, dEs, wsb)

    def timed(mode, steps, warmup):
        batch.set_launch_mode(mode)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    sec = timed(qfuse.QF_LAUNCH_GRAPH, args.steps, args.warmup)
    out = {
        "metric": "samples/s fwd+adjoint grad, 256 mixed circuits (10-18 qubits, 50-500 layers), one merged "
                  "HIP graph vs per-circuit launches",
        "value": round(n_samples / sec, 2), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1000 * sec, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "mixed256: 256 HEA circuits (RY,RZ + CZ ladder), qubits ~ U{10..18}, "
                               "layers ~ U{50..500}, 4 samples each, <Z_0>, L = sum E",
                   "circuits": len(ws), "samples": n_samples, "fwd_launches": int(info.fwd_launches),
                   "bwd_launches": int(info.bwd_launches), "fwd_jobs": int(info.fwd_jobs),
                   "bwd_jobs": int(info.bwd_jobs), "fwd_steps": int(info.fwd_steps),
                   "bwd_steps": int(info.bwd_steps), "uncompute": unc, "create_s": round(t_create, 2)},
    }
    flops = info.fwd_flops + info.bwd_flops
    byts = info.fwd_bytes + info.bwd_bytes
    out["roofline"] = {"kernel": "whole call (merged pass and small kernels)", "bound": "alu",
                       "achieved": round(flops / sec / 1e12, 2), "peak": round(PEAK_FP32_TFLOPS, 1),
                       "unit": "TFLOP/s", "frac": round(flops / sec / 1e12 / PEAK_FP32_TFLOPS, 4), "traffic": None,
                       "hbm_gbs": round(byts / sec / 1e9, 1)}
    if not args.no_baselines:
        sec_m = timed(qfuse.QF_LAUNCH_MERGED, 1, 1)
        sec_p = timed(qfuse.QF_LAUNCH_PER_CIRCUIT, 1, 1)
        out["merged_eager"] = {"value": round(n_samples / sec_m, 2), "unit": "samples/s"}
        out["per_circuit"] = {"value": round(n_samples / sec_p, 2), "unit": "samples/s",
                              "speedup_graph": round(sec_p / sec, 2)}
        # CPU oracle on a stratified sample: 8 circuits spread over the cost order, all their
        # samples, the first layers of each (about cpu_seconds / 8 each), extrapolated in depth
        # and then by amplitudes x gates x samples to the whole batch
        from oracle.oracle import Oracle
        from paper_2603_02804_amd.workloads import hea_gates
        orc = Oracle()

        def cost(c):
            return float(2 ** c.n_qubits) * len(c.gates) * c.x.shape[0]

        order = sorted(range(len(ws)), key=lambda i: cost(ws[i]))
        pick = [order[int(round(q * (len(order) - 1) / 7))] for q in range(8)]
        spent, est, cost_pick = 0.0, 0.0, 0.0
        for i in pick:
            c = ws[i]
            n = c.n_qubits
            t1 = time.perf_counter()
            g1 = hea_gates(n, 1, ("RY", "RZ"))
            orc.backward(n, g1, c.theta[:2 * n], c.x, xm, zm, np.ones((c.x.shape[0], 1)))
            per_layer = max(time.perf_counter() - t1, 1e-4)
            Lt = int(max(1, min(c.n_layers, round(args.cpu_seconds / 8 / per_layer))))
            g = hea_gates(n, Lt, ("RY", "RZ"))
            t = time.perf_counter()
            orc.backward(n, g, c.theta[:2 * n * Lt], c.x, xm, zm, np.ones((c.x.shape[0], 1)))
            dt = time.perf_counter() - t
            spent += dt + per_layer
            est += dt * c.n_layers / Lt
            cost_pick += cost(c)
        total = est * sum(cost(c) for c in ws) / cost_pick
        out["cpu_baseline"] = {"value": round(n_samples / total, 4), "unit": "samples/s",
                               "cores": orc.num_threads, "kind": "oracle", "host": host_info(),
                               "sample": f"8 circuits spread over the cost order, all 4 samples, leading layers "
                                         f"({spent:.1f} s), extrapolated in depth and by amplitudes x gates"}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
