"""Autotuner: tile shape, fusion depth, checkpoint interval and micro-batch.

Memory model (Sec. 3.4, eq. mem_cap_pytorch and eq. mem_cap_proposed): with
gradient checkpointing over blocks of b layers of a d-layer circuit, a method
that keeps s state vectors per layer of the active block needs
    M(b) = (s b + d / b) M_sv,   minimised at b* = sqrt(d / s),
s = l_var + l_const for per-gate storage, ceil(l_var / m) for fused gates of m
rotations.  This build checkpoints segments of fused passes instead of layers:
with P passes, segments of c passes, a batch B whose checkpoints are kept and a
micro-batch mb recomputed at a time,
    states(c) = ceil(P / c) B + (c - 1) mb + 4 mb,
minimised near c* = sqrt(P B / mb); the exact byte count is the plan's
qf_workspace_size.  In the uncompute mode (the adjoint passes rebuild psi)
the (c - 1) mb term vanishes, and segments are kept to at most
UNCOMPUTE_MAX_SEGMENT passes, which bounds the float32 drift of the rebuilt
states, as long as the checkpoints fit.

Speed: for each candidate (tile qubits, register qubits, fusion depth) the tuner
builds a plan for a prefix of the gate list, times forward + backward with HIP
events, and scales by the gate count.  Results are cached in a JSON file keyed
by the circuit's shape and the device name.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
from typing import Optional, Sequence

import numpy as np

TUNED_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_configs.json")

# (tile qubits, register qubits) shapes with compiled kernels
TILE_SHAPES = ((12, 4), (13, 5), (11, 4), (10, 4))
FUSION_DEPTHS = (4, 6, 8, 10, 12, 16)
MICRO_BATCHES = (8, 16, 32, 64, 128, 256, 512, 1024)
# end-of-pass epoch thresholds tried besides the default (every partial epoch waits): none waits, half
EPOCH_FILLS = (-1, 2)


def paper_memory_bytes(stored_per_layer: float, d: int, b: float, m_sv: int) -> float:
    """(s b + d / b) M_sv."""
    return (stored_per_layer * b + d / b) * m_sv


def paper_optimal_block(stored_per_layer: float, d: int) -> float:
    return math.sqrt(d / stored_per_layer)


def plan_states(passes: int, ckpt: int, batch: int, micro_batch: int, store: bool = True,
                mem_save: bool = False, uncompute: bool = False) -> float:
    """States held by a plan's workspace: checkpoints + one segment of pass outputs + ping-pong buffers.

    In the memory-saving mode the segment's pass outputs are bfloat16 pairs, half a state each (Sec. 3.4:
    the stored-output coefficient of the memory model is halved).  In the uncompute mode the adjoint
    passes rebuild psi, so no pass outputs are stored."""
    segs = -(-passes // ckpt)
    kept = batch if store else micro_batch
    seg_states = 0 if uncompute else max(0, ckpt - 1) * micro_batch
    return segs * kept + (seg_states / 2 if mem_save else seg_states) + 4 * micro_batch


# Longest checkpoint segment of the uncompute mode: psi is rebuilt in float32
# through at most this many fused passes before it restarts from a checkpoint.
UNCOMPUTE_MAX_SEGMENT = 64


def optimal_ckpt(passes: int, batch: int, micro_batch: int, store: bool = True, mem_save: bool = False) -> int:
    kept = batch if store else micro_batch
    per = micro_batch / 2 if mem_save else micro_batch
    guess = max(1, int(round(math.sqrt(passes * kept / max(1e-9, per)))))
    best = min(range(max(1, guess // 2), min(passes, 2 * guess) + 1),
               key=lambda c: (plan_states(passes, c, batch, micro_batch, store, mem_save), c))
    return best


def uncompute_storage(passes: int, batch: int, micro_batch: int, state_bytes: int, budget: float):
    """(store_ckpt, ckpt_interval) of the uncompute mode: checkpoints for the whole batch every
    UNCOMPUTE_MAX_SEGMENT passes, or fewer segments until they fit, else checkpoints per micro-batch.

    The segment cap bounds the float32 drift of the rebuilt states only while checkpoints fit at
    that interval; under a tight budget the segments grow, up to one segment of all passes, whose
    drift is the worst case (measured at 20 qubits x 1000 layers, 253 passes: normwise gradient
    error 2.3e-5 against the oracle).  When nothing fits, the least-memory option is returned
    (checkpoints per micro-batch, one segment), as choose_storage does."""
    c = min(passes, UNCOMPUTE_MAX_SEGMENT)
    for store in (1, 0):
        for ck in range(c, passes + 1):
            if plan_states(passes, ck, batch, micro_batch, bool(store), False, True) * state_bytes <= budget:
                return store, ck
            if -(-passes // ck) == 1:
                break
    return 0, passes


def choose_storage(passes: int, batch: int, micro_batch: int, state_bytes: int, budget: float):
    """(store_ckpt, mem_save, ckpt_interval): the first of full-precision checkpoints for the whole batch,
    the same with bfloat16 pass outputs, per-micro-batch checkpoints, and those with bfloat16 pass
    outputs whose workspace fits the budget (the last one when none fits)."""
    options = ((1, 0), (1, 1), (0, 0), (0, 1))
    for store, mem_save in options:
        c = optimal_ckpt(passes, batch, micro_batch, bool(store), bool(mem_save))
        if plan_states(passes, c, batch, micro_batch, bool(store), bool(mem_save)) * state_bytes <= budget:
            return store, mem_save, c
    return 0, 1, optimal_ckpt(passes, batch, micro_batch, False, True)


def circuit_key(n_qubits: int, gates: np.ndarray, n_obs: int, batch: int, device: str) -> str:
    h = hashlib.sha256(np.ascontiguousarray(gates, dtype=np.int32)[:, :3].tobytes()).hexdigest()[:16]
    return f"n{n_qubits}-g{len(gates)}-{h}-k{n_obs}-b{batch}-{device}"


def device_key(dev=None) -> str:
    """Cache key of a GPU: its ISA name and compute-unit count (the marketing name
    that the runtime reports depends on the host's device-id tables)."""
    import torch

    p = torch.cuda.get_device_properties(dev if dev is not None else torch.device("cuda"))
    arch = getattr(p, "gcnArchName", "") or p.name.replace(" ", "_")
    return f"{arch.split(':')[0]}-cu{p.multi_processor_count}"


def _load_cache(path: str) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def cached_tuning(n_qubits, gates, n_obs, batch, device, path: str = TUNED_CACHE) -> Optional[dict]:
    return _load_cache(path).get(circuit_key(n_qubits, gates, n_obs, batch, device))


def autotune(n_qubits: int, gates, n_params: int, n_inputs: int, z_masks: Sequence[int], batch: int,
             budget_bytes: Optional[int] = None, prefix_gates: int = 6000, reps: int = 2,
             shapes=TILE_SHAPES, depths=FUSION_DEPTHS, micro_batches=MICRO_BATCHES, epoch_fills=EPOCH_FILLS,
             cache_path: Optional[str] = None, log=None) -> dict:
    """Times the candidates on the current GPU and returns the chosen tuning fields.

    Each candidate (tile shape, fusion depth, micro-batch) runs forward + backward
    of one micro-batch on a prefix of the gate list, with the adjoint passes
    rebuilding psi (uncompute); the time per sample is scaled by the gate count.
    The best one is then timed with the other end-of-pass epoch thresholds
    (epoch_fills), and the best of those with the recompute scheme.  For the
    recompute scheme the checkpoint interval then minimises the workspace of
    the full circuit (memory model above), keeping checkpoints for the whole batch
    when they fit the budget.
    """
    import torch

    from . import qfuse

    gates = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 5)
    dev = torch.device("cuda")
    name = device_key(dev)
    G = len(gates)
    pre = gates[: min(G, prefix_gates)]
    P_used = int(pre[:, 3].max()) + 1 if (pre[:, 3] >= 0).any() else 0
    theta = torch.rand(max(P_used, 1), device=dev) * 6.283
    rng = np.random.default_rng(0)
    results = []
    circ = qfuse.Circuit(n_qubits, pre, max(P_used, 1), n_inputs, z_masks)
    def measure(k, r, F, mb, fill=0, unc=1):
        """ms per sample of the full circuit, from forward + backward of one micro-batch on the prefix."""
        try:
            plan = qfuse.Plan(circ, mb, qfuse.make_tuning(tile_qubits=k, reg_qubits=r, fusion_depth=F,
                                                          micro_batch=mb, epoch_fill=fill, uncompute=unc))
        except qfuse.QFuseError:
            return None
        x = torch.tensor(rng.uniform(-3.14, 3.14, size=(mb, n_inputs)).astype(np.float32), device=dev) \
            if n_inputs else None
        ws = plan.new_workspace(dev)
        dE = torch.ones(mb, len(z_masks), device=dev)
        best = float("inf")
        for _ in range(reps + 1):
            s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record()
            plan.forward(theta, x, ws)
            plan.backward(theta, x, dE, ws)
            s1.record()
            torch.cuda.synchronize()
            best = min(best, s0.elapsed_time(s1))
        del ws, plan
        per_sample_full = best / mb * (G / len(pre))
        res = {"tile_qubits": k, "reg_qubits": r, "fusion_depth": F, "micro_batch": mb, "epoch_fill": fill,
               "uncompute": unc, "ms_per_sample": round(per_sample_full, 4)}
        if log:
            log(f"autotune k={k} r={r} F={F} mb={mb} fill={fill} uncompute={unc}: {per_sample_full:.3f} ms/sample")
        return res

    for (k, r) in shapes:
        if k > n_qubits and (k, r) != shapes[0]:
            continue
        for F in depths:
            for mb in sorted(set(min(m, batch) for m in micro_batches)):
                res = measure(k, r, F, mb)
                if res is not None:
                    results.append(res)
    # the end-of-pass epoch threshold, tried for the best grid point (it trades
    # epochs against passes, which depends on the entangler pattern); then the
    # recompute scheme for the best of those
    if results:
        b = min(results, key=lambda d: d["ms_per_sample"])
        for fill in epoch_fills:
            res = measure(b["tile_qubits"], b["reg_qubits"], b["fusion_depth"], b["micro_batch"], fill)
            if res is not None:
                results.append(res)
        b = min(results, key=lambda d: d["ms_per_sample"])
        res = measure(b["tile_qubits"], b["reg_qubits"], b["fusion_depth"], b["micro_batch"], b["epoch_fill"], 0)
        if res is not None:
            results.append(res)
    if not results:
        raise RuntimeError("no candidate tuning could be planned")
    best = min(results, key=lambda d: d["ms_per_sample"])
    out = {k: best[k] for k in ("tile_qubits", "reg_qubits", "fusion_depth", "micro_batch", "epoch_fill",
                                "uncompute")}
    # checkpoint interval from the memory model of the full circuit
    full = qfuse.Circuit(n_qubits, gates, n_params, n_inputs, z_masks)
    probe = qfuse.Plan(full, batch, qfuse.make_tuning(tile_qubits=out["tile_qubits"], reg_qubits=out["reg_qubits"],
                                                      fusion_depth=out["fusion_depth"],
                                                      micro_batch=out["micro_batch"],
                                                      epoch_fill=out["epoch_fill"]))
    passes = probe.info.fused_passes
    del probe
    # the candidates' workspaces stay in torch's cache otherwise and shrink the free memory
    torch.cuda.empty_cache()
    free = torch.cuda.mem_get_info()[0]
    budget = budget_bytes if budget_bytes is not None else int(0.85 * free)
    if out["uncompute"]:
        store, c = uncompute_storage(passes, batch, out["micro_batch"], 8 << n_qubits, budget)
        mem_save = 0
    else:
        store, mem_save, c = choose_storage(passes, batch, out["micro_batch"], 8 << n_qubits, budget)
    out.update({"ckpt_interval": c, "store_ckpt": store, "mem_save": mem_save, "candidates": results, "device": name,
                "passes": passes, "prefix_gates": len(pre)})
    if cache_path:
        cache = _load_cache(cache_path)
        cache[circuit_key(n_qubits, gates, len(z_masks), batch, name)] = out
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return out


def tuning_from(d: dict):
    from . import qfuse
    return qfuse.make_tuning(tile_qubits=d.get("tile_qubits", 0), reg_qubits=d.get("reg_qubits", 0),
                             fusion_depth=d.get("fusion_depth", 0), ckpt_interval=d.get("ckpt_interval", 0),
                             micro_batch=d.get("micro_batch", 0), store_ckpt=d.get("store_ckpt", -1),
                             mem_save=d.get("mem_save", 0), epoch_fill=d.get("epoch_fill", 0),
                             uncompute=d.get("uncompute", 0))


def main(argv=None) -> int:
    """Tunes a named workload on the current GPU and writes the cache file."""
    import argparse

    from .workloads import c2, c3, c4

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="hea20q1000l", choices=("hea20q1000l", "hea16q200l", "hea12q100l"))
    ap.add_argument("--out", default=TUNED_CACHE)
    args = ap.parse_args(argv)
    w = {"hea20q1000l": c4, "hea16q200l": c3, "hea12q100l": c2}[args.workload]()
    out = autotune(w.n_qubits, w.gates, w.n_params, w.n_inputs, w.zmask, w.batch, cache_path=args.out,
                   log=lambda m: print(m, flush=True))
    print(json.dumps({k: v for k, v in out.items() if k != "candidates"}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
