"""Python binding of the CPU oracle (``qfo.c``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg.  The GPU library never imports this module.

Inputs are float32 arrays from the seeded generators, promoted exactly to
float64 before the call; every computation inside runs in complex128.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqfo.so")
SRC_PATH = os.path.join(_HERE, "qfo.c")


def build(src: str = SRC_PATH, out: str = LIB_PATH, extra: tuple = ()) -> str:
    """Compile the oracle with gcc (OpenMP across samples / amplitudes)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", *extra, src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_dptr = ctypes.POINTER(ctypes.c_double)
_iptr = ctypes.POINTER(ctypes.c_int32)
_uptr = ctypes.POINTER(ctypes.c_uint64)


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


class Oracle:
    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise FileNotFoundError(f"oracle library not built: {path}")
        lib = ctypes.CDLL(path)
        lib.qfo_forward.restype = ctypes.c_int
        lib.qfo_forward.argtypes = [ctypes.c_int, ctypes.c_int, _iptr, ctypes.c_int, _dptr,
                                    ctypes.c_int, _dptr, ctypes.c_int, _dptr,
                                    ctypes.c_int, _uptr, _uptr, _dptr, _dptr]
        lib.qfo_backward.restype = ctypes.c_int
        lib.qfo_backward.argtypes = [ctypes.c_int, ctypes.c_int, _iptr, ctypes.c_int, _dptr,
                                     ctypes.c_int, _dptr, ctypes.c_int, _dptr,
                                     ctypes.c_int, _uptr, _uptr, _dptr, _dptr, _dptr, _dptr,
                                     ctypes.c_int]
        lib.qfo_num_threads.restype = ctypes.c_int
        lib.qfo_set_num_threads.argtypes = [ctypes.c_int]
        self.lib = lib
        self.path = path

    @property
    def num_threads(self) -> int:
        return int(self.lib.qfo_num_threads())

    def set_num_threads(self, t: int) -> None:
        self.lib.qfo_set_num_threads(int(t))

    @staticmethod
    def _prep(gates, theta, x, xmask, zmask, psi0):
        gates = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 5)
        theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.ndim == 1:
            x = x.reshape(1, -1)
        xmask = np.ascontiguousarray(xmask, dtype=np.uint64).reshape(-1)
        zmask = np.ascontiguousarray(zmask, dtype=np.uint64).reshape(-1)
        if psi0 is not None:
            psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
            psi0 = psi0.view(np.float64)
        return gates, theta, x, xmask, zmask, psi0

    def forward(self, n_qubits, gates, theta, x, xmask, zmask, psi0=None, return_state=False):
        """E[b, k]; optionally also the final states [B, 2^n] complex128."""
        gates, theta, x, xmask, zmask, psi0 = self._prep(gates, theta, x, xmask, zmask, psi0)
        B, F = x.shape
        K = len(zmask)
        E = np.zeros((B, K), dtype=np.float64)
        psi = np.zeros((B, 1 << n_qubits), dtype=np.complex128) if return_state else None
        rc = self.lib.qfo_forward(n_qubits, len(gates), _p(gates, _iptr), len(theta), _p(theta, _dptr),
                                  F, _p(x, _dptr), B, _p(psi0, _dptr), K,
                                  _p(xmask, _uptr), _p(zmask, _uptr), _p(E, _dptr),
                                  psi.view(np.float64).ctypes.data_as(_dptr) if psi is not None else None)
        if rc != 0:
            raise ValueError(f"qfo_forward failed with code {rc}")
        return (E, psi) if return_state else E

    def backward(self, n_qubits, gates, theta, x, xmask, zmask, dE, mode=0, psi0=None):
        """(E, dtheta, dx) for upstream gradients dE[b, k] = dL/dE_k(b)."""
        gates, theta, x, xmask, zmask, psi0 = self._prep(gates, theta, x, xmask, zmask, psi0)
        B, F = x.shape
        K = len(zmask)
        dE = np.ascontiguousarray(dE, dtype=np.float64).reshape(B, K)
        E = np.zeros((B, K), dtype=np.float64)
        dtheta = np.zeros(len(theta), dtype=np.float64)
        dx = np.zeros((B, F), dtype=np.float64)
        rc = self.lib.qfo_backward(n_qubits, len(gates), _p(gates, _iptr), len(theta), _p(theta, _dptr),
                                   F, _p(x, _dptr), B, _p(psi0, _dptr), K,
                                   _p(xmask, _uptr), _p(zmask, _uptr), _p(dE, _dptr),
                                   _p(dtheta, _dptr), _p(dx, _dptr), _p(E, _dptr), int(mode))
        if rc != 0:
            raise ValueError(f"qfo_backward failed with code {rc}")
        return E, dtheta, dx


def loss_and_grad_E(E: np.ndarray, loss: str, labels: np.ndarray | None = None):
    """Loss of the expectations and dL/dE in float64 (the readings of the loss).

    sum:      L = sum_b sum_k E[b,k]                    (paper: L = E summed over the batch)
    mean_sum: L = sum_b mean_k E[b,k]
    ce:       L = mean_b CE(softmax(E[b]), label_b), logits = E unscaled
    """
    E = np.asarray(E, dtype=np.float64)
    B, K = E.shape
    if loss == "sum":
        return float(E.sum()), np.ones_like(E)
    if loss == "mean_sum":
        return float(E.mean(axis=1).sum()), np.full_like(E, 1.0 / K)
    if loss == "ce":
        m = E.max(axis=1, keepdims=True)
        ex = np.exp(E - m)
        p = ex / ex.sum(axis=1, keepdims=True)
        lab = np.asarray(labels, dtype=np.int64)
        L = float(-np.log(p[np.arange(B), lab]).mean())
        g = p.copy()
        g[np.arange(B), lab] -= 1.0
        return L, g / B
    raise ValueError(loss)
