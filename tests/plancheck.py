"""ctypes binding of the test-only CPU schedule checker (libqfuse_plancheck.so)."""
import ctypes
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_02804_amd", "libqfuse_plancheck.so")


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("theta_idx", ctypes.c_int32), ("input_idx", ctypes.c_int32)]


class Pauli(ctypes.Structure):
    _fields_ = [("x_mask", ctypes.c_uint64), ("z_mask", ctypes.c_uint64)]


class Desc(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_params", ctypes.c_int32), ("n_inputs", ctypes.c_int32),
                ("gates", ctypes.c_void_p), ("n_gates", ctypes.c_int64), ("obs", ctypes.c_void_p),
                ("n_obs", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("mode", "tile_qubits", "reg_qubits", "fusion_depth",
                                              "ckpt_interval", "micro_batch", "store_ckpt", "mem_save",
                                              "epoch_fill", "uncompute")]


def make_tuning(**kw):
    t = Tuning(0, 0, 0, 0, 0, 0, -1, 0, 0, 0)
    for k, v in kw.items():
        setattr(t, k, v)
    return t


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(LIB)
        _lib.qfc_last_error.restype = ctypes.c_char_p
    return _lib


def _desc(n, gates, n_params, n_inputs, zmask, xmask=None):
    gates = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 5)
    obs = np.zeros((len(zmask), 2), dtype=np.uint64)
    obs[:, 1] = np.asarray(zmask, dtype=np.uint64)
    if xmask is not None:
        obs[:, 0] = np.asarray(xmask, dtype=np.uint64)
    d = Desc(n, n_params, n_inputs, gates.ctypes.data, len(gates), obs.ctypes.data, len(zmask))
    return d, (gates, obs)


def run(n, gates, theta, x, zmask, dE=None, xmask=None, psi0=None, **tuning):
    theta = np.ascontiguousarray(theta, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    B = x.shape[0]
    K = len(zmask)
    d, keep = _desc(n, gates, len(theta), x.shape[1], zmask, xmask)
    t = make_tuning(**tuning)
    E = np.zeros((B, K), dtype=np.float32)
    dth = np.zeros(len(theta), dtype=np.float32)
    dx = np.zeros_like(x)
    f = ctypes.c_void_p
    dEa = None if dE is None else np.ascontiguousarray(dE, dtype=np.float32)
    p0 = None if psi0 is None else np.ascontiguousarray(psi0, dtype=np.complex64)
    rc = lib().qfc_run_psi0(ctypes.byref(d), B, ctypes.byref(t), f(theta.ctypes.data), f(x.ctypes.data),
                            f(p0.ctypes.data) if p0 is not None else None,
                            f(dEa.ctypes.data) if dEa is not None else None, f(E.ctypes.data), f(dth.ctypes.data),
                            f(dx.ctypes.data))
    if rc != 0:
        raise RuntimeError(f"qfc_run: {rc} {lib().qfc_last_error().decode()}")
    return E, dth, dx


def stats(n, gates, n_params, n_inputs, zmask, batch, **tuning):
    d, keep = _desc(n, gates, n_params, n_inputs, zmask)
    t = make_tuning(**tuning)
    out = (ctypes.c_int64 * 17)()
    rc = lib().qfc_stats(ctypes.byref(d), batch, ctypes.byref(t), out, 17)
    if rc != 0:
        raise RuntimeError(f"qfc_stats: {rc} {lib().qfc_last_error().decode()}")
    keys = ["passes", "segments", "ckpt", "micro_batch", "perm", "u2", "cz", "layouts", "runs", "k", "R", "ws_bytes",
            "diag_thread", "diag_amp", "threads", "thread_bits", "lds_bank_degree"]
    return dict(zip(keys, list(out)))


def batch_run(circuits, samples, thetas, xs, dEs=None, **tuning):
    """Mixed batch through the checker.  circuits: (n, gates, n_params, n_inputs, zmask) per circuit.

    Returns (Es, dthetas, dxs, stats)."""
    n = len(circuits)
    keep = []
    descs = (ctypes.c_void_p * n)()
    for i, (nq, gates, P, F, zm) in enumerate(circuits):
        d, k = _desc(nq, gates, P, F, zm)
        keep.append((d, k))
        descs[i] = ctypes.addressof(d)
    th = [np.ascontiguousarray(t, dtype=np.float32) for t in thetas]
    xx = [np.ascontiguousarray(x, dtype=np.float32) for x in xs]
    Es = [np.zeros((s, len(c[4])), dtype=np.float32) for c, s in zip(circuits, samples)]
    dth = [np.zeros(len(t), dtype=np.float32) for t in th]
    dxs = [np.zeros_like(x) for x in xx]
    dd = None if dEs is None else [np.ascontiguousarray(d, dtype=np.float32) for d in dEs]

    def arr(lst):
        a = (ctypes.c_void_p * n)()
        for i, v in enumerate(lst):
            a[i] = v.ctypes.data if v is not None and v.size else None
        return a

    t = make_tuning(**tuning)
    stats = (ctypes.c_int64 * 8)()
    ss = (ctypes.c_int32 * n)(*[int(s) for s in samples])
    rc = lib().qfc_batch_run(descs, ss, n, ctypes.byref(t), arr(th), arr(xx), arr(dd) if dd is not None else None,
                             arr(Es), arr(dth), arr(dxs), stats)
    if rc != 0:
        raise RuntimeError(f"qfc_batch_run: {rc} {lib().qfc_last_error().decode()}")
    keys = ["fwd_steps", "bwd_steps", "fwd_launches", "bwd_launches", "fwd_jobs", "bwd_jobs", "ws_bytes",
            "max_jobs_per_launch"]
    return Es, dth, dxs, dict(zip(keys, list(stats)))
