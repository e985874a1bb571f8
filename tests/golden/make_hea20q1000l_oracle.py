"""Writes tests/golden/hea20q1000l_oracle_2samples.npz with the CPU oracle only.

Workload: the 20-qubit, 1000-layer HEA (RX,RY,RZ + CZ ladder, RY encoding of 20
features, <Z_0..Z_9>, 10-class cross-entropy over a batch of 1000), drawn from
its seed.  For samples 0 and 1 it stores, in float64:
  E[2,10]              expectations;
  dE[2,10]             dL/dE of the mean cross-entropy over the full batch of
                       1000 (computed from these E and the labels);
  dtheta[60000]        dL/dtheta summed over the two samples;
  dx[2,20]             dL/dx per sample.
Runtime: about 10 minutes per sample on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, build  # noqa: E402
from paper_2603_02804_amd.workloads import c4  # noqa: E402

OUT = os.path.join(HERE, "hea20q1000l_oracle_2samples.npz")


def main():
    w = c4()
    orc = Oracle() if os.path.exists(os.path.join(ROOT, "oracle", "libqfo.so")) else Oracle(build())
    idx = [0, 1]
    x = w.x[idx]
    t0 = time.time()
    E = orc.forward(w.n_qubits, w.gates, w.theta, x, w.xmask, w.zmask)
    m = E.max(axis=1, keepdims=True)
    p = np.exp(E - m)
    p /= p.sum(axis=1, keepdims=True)
    dE = p.copy()
    dE[np.arange(2), w.labels[idx]] -= 1.0
    dE /= w.batch
    E2, dth, dx = orc.backward(w.n_qubits, w.gates, w.theta, x, w.xmask, w.zmask, dE)
    assert np.allclose(E, E2, atol=1e-12)
    np.savez(OUT, E=E, dE=dE, dtheta=dth, dx=dx, samples=np.asarray(idx), seconds=time.time() - t0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
