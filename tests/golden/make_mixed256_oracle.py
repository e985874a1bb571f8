"""Writes tests/golden/mixed256_oracle.npz with the CPU oracle only.

Workload: the mixed batch of 256 HEA circuits (qubits ~ U{10..18}, layers ~
U{50..500}, RY,RZ + CZ ladder, RY encoding, 4 samples each, <Z_0>), drawn from
its seed.  Eight circuits are taken spread evenly over the cost order
(2^n x gates x samples), the costliest included.  For each, in float64, with
L = sum over samples of <Z_0> (dL/dE = 1):
  E_<i>[4,1]         expectations;
  dtheta_<i>[P_i]    dL/dtheta summed over the circuit's 4 samples;
  dx_<i>[4,n_i]      dL/dx per sample.
`circuits` holds the chosen indices.  Runtime: about ten minutes on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, build  # noqa: E402
from paper_2603_02804_amd.workloads import c5, z_observables  # noqa: E402

OUT = os.path.join(HERE, "mixed256_oracle.npz")


def chosen(ws, k=8):
    cost = [float(2 ** c.n_qubits) * len(c.gates) * c.x.shape[0] for c in ws]
    order = sorted(range(len(ws)), key=lambda i: cost[i])
    return [order[int(round(q * (len(order) - 1) / (k - 1)))] for q in range(k)]


def main():
    ws = c5()
    orc = Oracle() if os.path.exists(os.path.join(ROOT, "oracle", "libqfo.so")) else Oracle(build())
    xm, zm = z_observables([0])
    out = {}
    idx = chosen(ws)
    t0 = time.time()
    for i in idx:
        c = ws[i]
        dE = np.ones((c.x.shape[0], 1))
        E, dth, dx = orc.backward(c.n_qubits, c.gates, c.theta, c.x, xm, zm, dE)
        out[f"E_{i}"], out[f"dtheta_{i}"], out[f"dx_{i}"] = E, dth, dx
        print(f"circuit {i}: {c.n_qubits} qubits, {c.n_layers} layers, {time.time() - t0:.0f} s", flush=True)
    np.savez(OUT, circuits=np.asarray(idx), **out)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
