"""Seeded synthetic workloads: HEA gate lists, angles, inputs, labels, observables.

This module only builds inputs.  It holds none of the simulation's arithmetic and
is shared by the GPU path, the CPU oracle and the benchmark, so both sides of
every parity check see identical inputs.

Circuit shape (paper Sec. 4.2, Fig. "HEA"): each layer applies the listed Pauli
rotations to every qubit, then CZ gates between neighbouring qubits.  The paper's
20-qubit layer has 60 rotations and 20 CZ gates (App. C), i.e. a closed ring; the
benchmark configurations here use an open ladder (q, q+1), q = 0..n-2, and a ring
is available as an option.  Inputs are angle-encoded by RY(x_q) on qubit q before
the first layer.

Gate rows are int32 quintuples ``(kind, q0, q1, theta_idx, input_idx)`` with
kind 0=RX, 1=RY, 2=RZ, 3=CZ, 4=CNOT (q0 control, q1 target).  A rotation takes its angle from ``theta[theta_idx]``
when ``theta_idx >= 0`` and from ``x[b, input_idx]`` otherwise.

Random draws follow one fixed recipe: ``numpy.random.default_rng(seed)``, then
theta ~ U[0, 2 pi), x ~ U[-pi, pi], labels ~ U{0..K-1}, in that order, as float32.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np

RX, RY, RZ, CZ, CNOT = 0, 1, 2, 3, 4
_ROT_CODES = {"RX": RX, "RY": RY, "RZ": RZ}


def hea_gates(n_qubits: int, n_layers: int, rotations: Sequence[str] = ("RY", "RZ"),
              encoding: bool = True, ring: bool = False, entangler: int = CZ) -> np.ndarray:
    """Gate list of an HEA with optional RY input encoding; the entangling ladder
    (or ring) uses CZ, or CNOT(q -> q+1) with ``entangler=CNOT``.

    Parameter index of layer l, rotation r, qubit q: ``l * (R * n) + r * n + q``.
    """
    rows = []
    if encoding:
        for q in range(n_qubits):
            rows.append((RY, q, -1, -1, q))
    R = len(rotations)
    for layer in range(n_layers):
        for r, name in enumerate(rotations):
            code = _ROT_CODES[name]
            for q in range(n_qubits):
                rows.append((code, q, -1, layer * R * n_qubits + r * n_qubits + q, -1))
        for q in range(n_qubits - 1):
            rows.append((entangler, q, q + 1, -1, -1))
        if ring and n_qubits > 2:
            rows.append((entangler, n_qubits - 1, 0, -1, -1))
    return np.asarray(rows, dtype=np.int32).reshape(-1, 5)


def z_observables(qubits: Sequence[int]) -> tuple[np.ndarray, np.ndarray]:
    """Single-qubit Z observables: (x_masks, z_masks) as uint64 arrays."""
    z = np.asarray([1 << int(q) for q in qubits], dtype=np.uint64)
    return np.zeros_like(z), z


def pauli_string(spec: str) -> tuple[int, int]:
    """Masks of a Pauli string; the rightmost character acts on qubit 0."""
    xm = zm = 0
    for q, ch in enumerate(reversed(spec)):
        if ch in "XY":
            xm |= 1 << q
        if ch in "ZY":
            zm |= 1 << q
        if ch not in "IXYZ":
            raise ValueError(f"bad Pauli character {ch!r}")
    return xm, zm


def draw_inputs(seed: int, n_params: int, batch: int, n_inputs: int, n_labels: int = 0):
    """theta ~ U[0,2pi), x ~ U[-pi,pi], labels ~ U{0..n_labels-1}; float32 / int64."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * math.pi, size=n_params).astype(np.float32)
    x = rng.uniform(-math.pi, math.pi, size=(batch, n_inputs)).astype(np.float32)
    labels = (rng.integers(0, n_labels, size=batch).astype(np.int64)
              if n_labels > 0 else np.zeros(batch, dtype=np.int64))
    return theta, x, labels


@dataclasses.dataclass
class Workload:
    """One benchmark configuration, fully materialised from its seed."""
    name: str
    n_qubits: int
    n_layers: int
    rotations: tuple
    batch: int
    obs_qubits: tuple
    loss: str              # "sum" | "mean_sum" | "ce"
    seed: int
    gates: np.ndarray = None
    theta: np.ndarray = None
    x: np.ndarray = None
    labels: np.ndarray = None
    xmask: np.ndarray = None
    zmask: np.ndarray = None

    @property
    def n_params(self) -> int:
        return self.n_layers * len(self.rotations) * self.n_qubits

    @property
    def n_inputs(self) -> int:
        return self.n_qubits

    @property
    def n_obs(self) -> int:
        return len(self.obs_qubits)


def make_workload(name: str, n_qubits: int, n_layers: int, rotations, batch: int,
                  obs_qubits, loss: str, seed: int, batch_override: int | None = None) -> Workload:
    w = Workload(name, n_qubits, n_layers, tuple(rotations), batch, tuple(obs_qubits), loss, seed)
    w.gates = hea_gates(n_qubits, n_layers, rotations)
    n_labels = len(obs_qubits) if loss == "ce" else 0
    w.theta, w.x, w.labels = draw_inputs(seed, w.n_params, batch, n_qubits, n_labels)
    if batch_override is not None:
        w.batch = batch_override
        w.x = w.x[:batch_override].copy()
        w.labels = w.labels[:batch_override].copy()
    w.xmask, w.zmask = z_observables(obs_qubits)
    return w


# The five configurations.  Seeds: C1=1 ... C5=5.
def c1(**kw) -> Workload:
    """4-qubit HEA, 2 layers (RY,RZ + CZ ladder), RY encoding, batch 8, <Z_0>, L = sum_b E."""
    return make_workload("hea4q2l", 4, 2, ("RY", "RZ"), 8, (0,), "sum", 1, **kw)


def c2(**kw) -> Workload:
    """12-qubit HEA, 100 layers (RY,RZ + ladder), batch 1024, mean_i <Z_i>."""
    return make_workload("hea12q100l", 12, 100, ("RY", "RZ"), 1024, tuple(range(12)), "mean_sum", 2, **kw)


def c3(**kw) -> Workload:
    """16-qubit HEA, 200 layers (RX,RY,RZ + ladder), batch 512, <Z_0..Z_3> -> 4-class CE."""
    return make_workload("hea16q200l", 16, 200, ("RX", "RY", "RZ"), 512, (0, 1, 2, 3), "ce", 3, **kw)


def c4(**kw) -> Workload:
    """20-qubit HEA, 1000 layers (RX,RY,RZ + ladder), batch 1000, <Z_0..Z_9> -> 10-class CE."""
    return make_workload("hea20q1000l", 20, 1000, ("RX", "RY", "RZ"), 1000, tuple(range(10)), "ce", 4, **kw)


@dataclasses.dataclass
class MixedCircuit:
    n_qubits: int
    n_layers: int
    gates: np.ndarray
    theta: np.ndarray
    x: np.ndarray


def mixed(n_circuits: int, qubits=(10, 18), layers=(50, 500), samples: int = 4, seed: int = 5,
          rotations=("RY", "RZ")):
    """Mixed batch: qubits ~ U{qubits}, layers ~ U{layers} (inclusive), HEA + ladder, <Z_0>.

    Draw order: for the whole set, qubit counts then layer counts; then per
    circuit theta ~ U[0,2pi) and x ~ U[-pi,pi]^(samples x n).
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(qubits[0], qubits[1] + 1, size=n_circuits)
    ls = rng.integers(layers[0], layers[1] + 1, size=n_circuits)
    out = []
    for n, L in zip(ns.tolist(), ls.tolist()):
        theta = rng.uniform(0.0, 2.0 * math.pi, size=len(rotations) * n * L).astype(np.float32)
        x = rng.uniform(-math.pi, math.pi, size=(samples, n)).astype(np.float32)
        out.append(MixedCircuit(n, L, hea_gates(n, L, rotations), theta, x))
    return out


def c5(n_circuits: int = 256, samples: int = 4, seed: int = 5):
    """256 circuits, qubits ~ U{10..18}, layers ~ U{50..500}, RY,RZ + ladder, 4 samples each, <Z_0>."""
    return mixed(n_circuits, (10, 18), (50, 500), samples, seed)


@dataclasses.dataclass
class PaperModeWorkload:
    """The paper's own experiment shape (Sec. 4): random initial states, an HEA of
    RX, RY, RZ layers closed into a CZ ring, and the observable (IXYZ) repeated
    over the register."""
    n_qubits: int
    n_layers: int
    gates: np.ndarray
    theta: np.ndarray
    psi0: np.ndarray         # complex64 [batch, 2^n], unit norm per sample
    xmask: np.ndarray
    zmask: np.ndarray


def paper_mode(n_qubits: int, n_layers: int, batch: int, seed: int = 6) -> PaperModeWorkload:
    """Seeded paper-mode inputs: theta ~ U[0, 2 pi) as float32, then psi0 with
    independent standard normal real and imaginary parts, normalised per sample
    (the paper does not state its distribution; this is the reading taken)."""
    gates = hea_gates(n_qubits, n_layers, ("RX", "RY", "RZ"), encoding=False, ring=n_qubits > 2)
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * math.pi, n_layers * 3 * n_qubits).astype(np.float32)
    psi = rng.standard_normal((batch, 1 << n_qubits)) + 1j * rng.standard_normal((batch, 1 << n_qubits))
    psi /= np.linalg.norm(psi, axis=1, keepdims=True)
    spec = ("IXYZ" * (n_qubits // 4 + 1))[:n_qubits]
    xm, zm = pauli_string(spec)
    return PaperModeWorkload(n_qubits, n_layers, gates, theta, psi.astype(np.complex64),
                             np.array([xm], np.uint64), np.array([zm], np.uint64))
