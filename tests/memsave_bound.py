"""Error bound of the memory-saving mode (Sec. 3.2, Sec. 3.4), shared by its CPU
and GPU tests.

In that mode each stored pass output is rounded once to bfloat16 pairs, so the
state the adjoint pass starts from carries ||dpsi|| <= 2^-8 ||psi|| (half an ulp
of an 8-bit significand per component).  Un-applying runs is unitary and keeps
that norm.  The functionals F_P = Im<lambda|P|psi> then move by at most
||lambda|| ||dpsi||, and a gate's gradient 1/2 n.F (n a unit vector: the gate's
generator carried to the cut) by at most 1/2 sqrt(3) 2^-8 ||lambda||.  lambda is
not affected (the seed is formed from the float32 final state), and
||lambda_b|| = 2 ||sum_k g_bk O_k psi_b|| is computed here from the oracle's
final states.
"""
import numpy as np

STEP = 0.5 * np.sqrt(3.0) * 2.0 ** -8


def lambda_norms(orc, n, gates, theta, x, zmask, dE):
    """||lambda_M|| per sample for Z-string observables."""
    _, psi = orc.forward(n, gates, theta, x, np.zeros(len(zmask), np.uint64), zmask, return_state=True)
    idx = np.arange(1 << n, dtype=np.uint64)
    signs = np.stack([1.0 - 2.0 * (np.bitwise_count(idx & np.uint64(z)) & 1) for z in zmask])   # K x 2^n
    c = np.asarray(dE, np.float64) @ signs                                                         # B x 2^n
    return 2.0 * np.sqrt(np.sum(np.abs(psi) ** 2 * c ** 2, axis=1))


def gradient_bounds(gates, n_params, n_inputs, lam):
    """Largest change of dL/dtheta (summed over samples) and dL/dx the rounding can cause."""
    g = np.asarray(gates)
    rot = g[:, 0] != 3
    th_uses = np.bincount(g[rot & (g[:, 3] >= 0), 3], minlength=n_params)[:n_params]
    in_uses = np.bincount(g[rot & (g[:, 4] >= 0), 4], minlength=n_inputs)[:n_inputs]
    dth = STEP * th_uses * lam.sum()
    dx = STEP * np.outer(lam, in_uses)
    return dth, dx
