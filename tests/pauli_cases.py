"""Observable sets for the Pauli-string tests (shared by the CPU and GPU tests)."""
import numpy as np

from paper_2603_02804_amd.workloads import pauli_string


def strings(n):
    """Single X / Y / Z on low, middle and top qubits, two-qubit strings across
    the tile boundary, and (IXYZ) repeated over the register."""
    out = [("Z", 0), ("X", n - 1), ("Y", n // 2), ("XX", (0, n - 1)), ("YZ", (3, n - 2))]
    masks = []
    for kind, q in out:
        qs = (q,) if isinstance(q, int) else q
        spec = ["I"] * n
        for ch, qq in zip(kind, qs):
            spec[n - 1 - qq] = ch
        masks.append(pauli_string("".join(spec)))
    rep = ("IXYZ" * (n // 4 + 1))[:n]
    masks.append(pauli_string(rep))
    xm = np.array([m[0] for m in masks], np.uint64)
    zm = np.array([m[1] for m in masks], np.uint64)
    return xm, zm
