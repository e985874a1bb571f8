"""Pins for the CPU oracle: checks against facts fixed by the paper and by mathematics.

Each pin takes an ``Oracle`` and raises ``AssertionError`` on a mismatch.  The
same pins run against the real oracle (tests/test_oracle.py) and against
mutated copies of it (tests/test_oracle_mutants.py), which shows that a
plausible mistake anywhere in the oracle fails at least one of them.

Sources of truth (none is the oracle itself):
  P1  one-qubit closed forms of u(phi) = cos(phi/2) I - i sin(phi/2) P   (Sec. 3.3)
  P2  a two-qubit closed form with CZ, and its three derivatives          (Sec. 3.1)
  P3  all variational angles zero: <Z_i> = cos x_i, dL/dx_i = -g_i sin x_i
  P4  norm preservation of every gate sequence
  P5  dense 2^n x 2^n products of Kronecker-embedded gates (qubit 0 rightmost)
  P6  parameter-shift rule, exact for exp(-i phi P / 2)                    (Sec. 1)
  P7  un-apply backward vs store-all backward vs central finite differences (Sec. 2.2)
  P9  Pauli-string expectation vs the dense Pauli product                 (App. B.2)
  P10 CNOT: the truth table on basis states, the Bell-state closed forms and the
      parameter shift through CNOT ladders (P5 and P6 also draw CNOT gates)
  P11 caller-supplied initial states: dense products from psi0, and the parameter
      shift of dense expectations from psi0                                (Sec. 4)
  L1  the loss readings (sum, mean over observables, mean cross-entropy) against
      closed forms, the two-class logistic special case, invariants and finite
      differences; these pins take the loss helper instead of the oracle library
"""
from __future__ import annotations

import math

import numpy as np

from paper_2603_02804_amd.workloads import CNOT, CZ, RX, RY, RZ, hea_gates, pauli_string, z_observables

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _g(kind, q0, q1=-1, t=-1, f=-1):
    return (kind, q0, q1, t, f)


def _gates(rows):
    return np.asarray(rows, dtype=np.int32).reshape(-1, 5)


def _E(orc, n, gates, theta, x, obs):
    xm = np.asarray([o[0] for o in obs], dtype=np.uint64)
    zm = np.asarray([o[1] for o in obs], dtype=np.uint64)
    return orc.forward(n, gates, theta, x, xm, zm)


# ---------------------------------------------------------------- P1
def pin_p1_single_qubit(orc):
    """RY(phi)|0>: <Z>=cos phi, <X>=sin phi.  RX(phi)|0>: <Z>=cos phi, <Y>=-sin phi.
    RZ(phi) after RY(a)|0> turns the Bloch vector about z: <X>=sin a cos phi,
    <Y>=sin a sin phi, <Z>=cos a.  u(phi) u(-phi) = I.  The adjoint backward of a
    single RX or RY gives d<Z>/dphi = -sin phi."""
    X, Y, Z = (1, 0), (1, 1), (0, 1)
    for phi in (0.3, 1.1, -2.4, 3.0):
        E = _E(orc, 1, _gates([_g(RY, 0, t=0)]), [phi], np.zeros((1, 0)), [Z, X, Y])[0]
        np.testing.assert_allclose(E, [math.cos(phi), math.sin(phi), 0.0], atol=1e-13)
        E = _E(orc, 1, _gates([_g(RX, 0, t=0)]), [phi], np.zeros((1, 0)), [Z, X, Y])[0]
        np.testing.assert_allclose(E, [math.cos(phi), 0.0, -math.sin(phi)], atol=1e-13)
        a = 0.7
        E = _E(orc, 1, _gates([_g(RY, 0, t=0), _g(RZ, 0, t=1)]), [a, phi], np.zeros((1, 0)), [Z, X, Y])[0]
        np.testing.assert_allclose(E, [math.cos(a), math.sin(a) * math.cos(phi), math.sin(a) * math.sin(phi)],
                                   atol=1e-13)
        # u(phi) u(-phi) = I for each Pauli: the state returns to RY(a)|0>
        for k in (RX, RY, RZ):
            E = _E(orc, 1, _gates([_g(RY, 0, t=0), _g(k, 0, t=1), _g(k, 0, t=2)]), [a, phi, -phi],
                   np.zeros((1, 0)), [Z, X, Y])[0]
            np.testing.assert_allclose(E, [math.cos(a), math.sin(a), 0.0], atol=1e-13)
        for k in (RX, RY):
            gates = _gates([_g(k, 0, t=0)])
            _, dth, _ = orc.backward(1, gates, [phi], np.zeros((1, 0)), [0], [1], [[1.0]])
            np.testing.assert_allclose(dth, [-math.sin(phi)], atol=1e-13)


# ---------------------------------------------------------------- P2
def pin_p2_two_qubit(orc):
    """RY(a) q0, RY(b) q1, CZ(0,1), RY(c) q0:  <Z_0> = cos a cos c - sin a sin c cos b.
    The angles a and b come from the input vector x, c from theta, so both gradient
    outputs are checked against the closed-form derivatives."""
    rng = np.random.default_rng(12)
    for _ in range(4):
        a, b, c = rng.uniform(-math.pi, math.pi, size=3)
        gates = _gates([_g(RY, 0, f=0), _g(RY, 1, f=1), _g(CZ, 0, 1), _g(RY, 0, t=0)])
        x = np.array([[a, b]])
        E, dth, dx = orc.backward(2, gates, [c], x, [0], [1], [[1.0]])
        ref = math.cos(a) * math.cos(c) - math.sin(a) * math.sin(c) * math.cos(b)
        np.testing.assert_allclose(E[0, 0], ref, atol=1e-13)
        da = -math.sin(a) * math.cos(c) - math.cos(a) * math.sin(c) * math.cos(b)
        db = math.sin(a) * math.sin(c) * math.sin(b)
        dc = -math.cos(a) * math.sin(c) - math.sin(a) * math.cos(c) * math.cos(b)
        np.testing.assert_allclose(dx[0], [da, db], atol=1e-13)
        np.testing.assert_allclose(dth, [dc], atol=1e-13)
        # the CZ order (control/target) does not matter
        gates2 = _gates([_g(RY, 0, f=0), _g(RY, 1, f=1), _g(CZ, 1, 0), _g(RY, 0, t=0)])
        E2 = orc.forward(2, gates2, [c], x, [0], [1])
        np.testing.assert_allclose(E2[0, 0], ref, atol=1e-13)


# ---------------------------------------------------------------- P3
def pin_p3_zero_angles(orc, n=7, layers=3):
    """All variational angles zero: the HEA reduces to the encoding plus diagonal
    gates, so <Z_i> = cos x_i and dL/dx_i = -g_i sin x_i (L = sum_i g_i <Z_i>)."""
    for rots in (("RY", "RZ"), ("RX", "RY", "RZ")):
        gates = hea_gates(n, layers, rots)
        P = layers * len(rots) * n
        rng = np.random.default_rng(3)
        x = rng.uniform(-math.pi, math.pi, size=(3, n))
        g = rng.normal(size=(3, n))
        xm, zm = z_observables(range(n))
        E, dth, dx = orc.backward(n, gates, np.zeros(P), x, xm, zm, g)
        np.testing.assert_allclose(E, np.cos(x), atol=1e-12)
        np.testing.assert_allclose(dx, -g * np.sin(x), atol=1e-12)
    # only RZ angles non-zero keeps the same expectations
    gates = hea_gates(n, layers, ("RY", "RZ"))
    theta = np.zeros(layers * 2 * n)
    for l in range(layers):
        theta[l * 2 * n + n: l * 2 * n + 2 * n] = np.linspace(0.3, 2.9, n)
    x = np.random.default_rng(4).uniform(-math.pi, math.pi, size=(2, n))
    xm, zm = z_observables(range(n))
    np.testing.assert_allclose(orc.forward(n, gates, theta, x, xm, zm), np.cos(x), atol=1e-12)


# ---------------------------------------------------------------- P4
def pin_p4_norm(orc, n=9, layers=6):
    gates = hea_gates(n, layers, ("RX", "RY", "RZ"))
    rng = np.random.default_rng(5)
    theta = rng.uniform(0, 2 * math.pi, size=layers * 3 * n)
    x = rng.uniform(-math.pi, math.pi, size=(4, n))
    xm, zm = z_observables([0])
    E, psi = orc.forward(n, gates, theta, x, xm, zm, return_state=True)
    np.testing.assert_allclose(np.sum(np.abs(psi) ** 2, axis=1), 1.0, atol=1e-12)
    assert np.all(np.abs(E) <= 1.0 + 1e-12)


# ---------------------------------------------------------------- P5
def _u_dense(kind, phi):
    P = {RX: PX, RY: PY, RZ: PZ}[kind]
    return math.cos(phi / 2) * I2 - 1j * math.sin(phi / 2) * P


def _embed(n, q, u):
    """Kronecker embedding; qubit 0 is the rightmost factor."""
    m = np.array([[1.0 + 0j]])
    for k in reversed(range(n)):
        m = np.kron(m, u if k == q else I2)
    return m


def _cz_dense(n, a, b):
    d = np.ones(1 << n, dtype=np.complex128)
    for i in range(1 << n):
        if (i >> a) & 1 and (i >> b) & 1:
            d[i] = -1
    return np.diag(d)


def _cnot_dense(n, c, t):
    """The permutation matrix of CNOT: |x> -> |x ^ 2^t> where bit c of x is 1."""
    m = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for i in range(1 << n):
        j = i ^ (1 << t) if (i >> c) & 1 else i
        m[j, i] = 1
    return m


def dense_state(n, gates, theta, xb, psi0=None):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    if psi0 is not None:
        psi = np.asarray(psi0, dtype=np.complex128).copy()
    U = np.eye(1 << n, dtype=np.complex128)
    for (k, q0, q1, t, f) in gates:
        if k == CZ:
            G = _cz_dense(n, q0, q1)
        elif k == CNOT:
            G = _cnot_dense(n, q0, q1)
        else:
            phi = theta[t] if t >= 0 else xb[f]
            G = _embed(n, q0, _u_dense(k, phi))
        U = G @ U
    return U @ psi


def pin_p5_dense(orc):
    rng = np.random.default_rng(6)
    for n in (1, 2, 3, 5, 6):
        rows = []
        t = 0
        for _ in range(4 * n + 3):
            k = int(rng.integers(0, 5)) if n > 1 else int(rng.integers(0, 3))
            q0 = int(rng.integers(0, n))
            if k in (CZ, CNOT):
                q1 = int((q0 + 1 + rng.integers(0, n - 1)) % n)
                rows.append(_g(k, q0, q1))
            elif rng.random() < 0.3:
                rows.append(_g(k, q0, f=int(rng.integers(0, n))))
            else:
                rows.append(_g(k, q0, t=t))
                t += 1
        gates = _gates(rows)
        theta = rng.uniform(0, 2 * math.pi, size=max(t, 1))
        x = rng.uniform(-math.pi, math.pi, size=(2, n))
        xm, zm = z_observables([0])
        _, psi = orc.forward(n, gates, theta, x, xm, zm, return_state=True)
        for b in range(2):
            np.testing.assert_allclose(psi[b], dense_state(n, gates, theta, x[b]), atol=1e-12)


# ---------------------------------------------------------------- P6
def pin_p6_parameter_shift(orc, n=6, layers=4):
    """dE/dphi = [E(phi + pi/2) - E(phi - pi/2)] / 2 for every gate angle."""
    gates = hea_gates(n, layers, ("RX", "RY", "RZ"))
    rng = np.random.default_rng(7)
    P = layers * 3 * n
    theta = rng.uniform(0, 2 * math.pi, size=P)
    x = rng.uniform(-math.pi, math.pi, size=(1, n))
    xm, zm = z_observables([0, 2, 5])
    g = np.array([[0.7, -1.3, 0.4]])
    _, dth, dx = orc.backward(n, gates, theta, x, xm, zm, g)

    def L(th, xx):
        return float((orc.forward(n, gates, th, xx, xm, zm) * g).sum())

    for p in list(range(0, P, 7)) + [P - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += math.pi / 2
        tm[p] -= math.pi / 2
        np.testing.assert_allclose(dth[p], 0.5 * (L(tp, x) - L(tm, x)), atol=1e-11)
    for f in range(n):
        xp, xmn = x.copy(), x.copy()
        xp[0, f] += math.pi / 2
        xmn[0, f] -= math.pi / 2
        np.testing.assert_allclose(dx[0, f], 0.5 * (L(theta, xp) - L(theta, xmn)), atol=1e-11)


# ---------------------------------------------------------------- P7
def pin_p7_backward_modes(orc, n=5, layers=3):
    """Un-apply backward == store-all backward == central finite differences;
    a shared angle (used by two gates) receives the sum of both contributions."""
    gates = hea_gates(n, layers, ("RY", "RZ"))
    rows = [tuple(r) for r in gates.tolist()]
    rows.append(_g(RX, 0, t=0))          # theta[0] drives two gates
    rows.append(_g(RY, 3, f=1))          # x[:, 1] drives two gates
    gates = _gates(rows)
    rng = np.random.default_rng(8)
    P = layers * 2 * n
    theta = rng.uniform(0, 2 * math.pi, size=P)
    x = rng.uniform(-math.pi, math.pi, size=(3, n))
    xm, zm = z_observables([0, 3])
    g = rng.normal(size=(3, 2))
    E0, d0, x0 = orc.backward(n, gates, theta, x, xm, zm, g, mode=0)
    E1, d1, x1 = orc.backward(n, gates, theta, x, xm, zm, g, mode=1)
    np.testing.assert_allclose(d0, d1, atol=1e-12)
    np.testing.assert_allclose(x0, x1, atol=1e-12)
    np.testing.assert_allclose(E0, E1, atol=1e-13)

    def L(th, xx):
        return float((orc.forward(n, gates, th, xx, xm, zm) * g).sum())

    h = 1e-5
    for p in range(P):
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        np.testing.assert_allclose(d0[p], (L(tp, x) - L(tm, x)) / (2 * h), atol=1e-8)
    for b in range(3):
        for f in range(n):
            xp, xmn = x.copy(), x.copy()
            xp[b, f] += h
            xmn[b, f] -= h
            np.testing.assert_allclose(x0[b, f], (L(theta, xp) - L(theta, xmn)) / (2 * h), atol=1e-8)


# ---------------------------------------------------------------- P9
def _pauli_dense(spec):
    m = np.array([[1.0 + 0j]])
    for ch in spec:          # leftmost character = highest qubit
        m = np.kron(m, {"I": I2, "X": PX, "Y": PY, "Z": PZ}[ch])
    return m


def pin_p9_pauli_expectation(orc, n=5):
    rng = np.random.default_rng(9)
    gates = hea_gates(n, 2, ("RX", "RY", "RZ"))
    theta = rng.uniform(0, 2 * math.pi, size=2 * 3 * n)
    x = rng.uniform(-math.pi, math.pi, size=(2, n))
    specs = ["IXYZI", "ZZZZZ", "YYIXX", "XIIIY", "IIIIZ", "YIIII"]
    masks = [pauli_string(s) for s in specs]
    xm = np.asarray([m[0] for m in masks], dtype=np.uint64)
    zm = np.asarray([m[1] for m in masks], dtype=np.uint64)
    E, psi = orc.forward(n, gates, theta, x, xm, zm, return_state=True)
    for b in range(2):
        for k, s in enumerate(specs):
            ref = np.vdot(psi[b], _pauli_dense(s) @ psi[b]).real
            np.testing.assert_allclose(E[b, k], ref, atol=1e-12)
    # the adjoint seed with a general Pauli string agrees with finite differences
    g = rng.normal(size=(2, len(specs)))
    _, d0, _ = orc.backward(n, gates, theta, x, xm, zm, g)
    h = 1e-5
    for p in (0, 5, 17, 29):
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd = ((orc.forward(n, gates, tp, x, xm, zm) - orc.forward(n, gates, tm, x, xm, zm)) * g).sum() / (2 * h)
        np.testing.assert_allclose(d0[p], fd, atol=1e-8)


# ---------------------------------------------------------------- P10
def pin_p10_cnot(orc):
    """CNOT truth table; RY(a) on the control, then CNOT(0 -> 1): <Z_1> = cos a, <Z_0 Z_1> = 1,
    <X_0 X_1> = sin a; a parameter-shift check through a CNOT ladder."""
    n = 3
    for c, t in ((0, 1), (1, 0), (2, 0), (0, 2)):
        for basis in range(1 << n):
            # prepare |basis> with RX(pi) flips, then CNOT
            rows = [_g(RX, q, t=0) for q in range(n) if (basis >> q) & 1] + [_g(CNOT, c, t)]
            _, psi = orc.forward(n, _gates(rows), np.array([math.pi]), np.zeros((1, 0)),
                                 np.zeros(1, np.uint64), np.array([1], np.uint64), return_state=True)
            out = basis ^ (1 << t) if (basis >> c) & 1 else basis
            assert abs(abs(psi[0][out]) - 1.0) < 1e-12
    for a in (0.3, 1.1, 2.9):
        gates = _gates([_g(RY, 0, t=0), _g(CNOT, 0, 1)])
        E = _E(orc, 2, gates, np.array([a]), np.zeros((1, 0)),
               [pauli_string("ZI"), pauli_string("ZZ"), pauli_string("XX"), pauli_string("IZ")])
        np.testing.assert_allclose(E[0], [math.cos(a), 1.0, math.sin(a), math.cos(a)], atol=1e-12)
    # parameter shift through a CNOT ladder, theta and x angles
    nq, L = 4, 2
    rows = [_g(RY, q, f=q) for q in range(nq)]
    t = 0
    for _ in range(L):
        for q in range(nq):
            rows.append(_g(RY, q, t=t))
            t += 1
        for q in range(nq - 1):
            rows.append(_g(CNOT, q, q + 1))
    gates = _gates(rows)
    rng = np.random.default_rng(10)
    theta = rng.uniform(0, 2 * math.pi, t)
    x = rng.uniform(-math.pi, math.pi, (1, nq))
    xm, zm = pauli_string("IIXZ")
    dE = np.array([[1.0]])
    _, dth, dx = orc.backward(nq, gates, theta, x, np.array([xm], np.uint64), np.array([zm], np.uint64), dE)
    for p in range(t):
        tp, tm = theta.copy(), theta.copy()
        tp[p] += math.pi / 2
        tm[p] -= math.pi / 2
        ep = orc.forward(nq, gates, tp, x, np.array([xm], np.uint64), np.array([zm], np.uint64))[0, 0]
        em = orc.forward(nq, gates, tm, x, np.array([xm], np.uint64), np.array([zm], np.uint64))[0, 0]
        assert abs(dth[p] - (ep - em) / 2) < 1e-10


# ---------------------------------------------------------------- P11
def _random_states(rng, B, n):
    psi = rng.standard_normal((B, 1 << n)) + 1j * rng.standard_normal((B, 1 << n))
    return psi / np.linalg.norm(psi, axis=1, keepdims=True)


def pin_p11_initial_states(orc):
    """Caller-supplied initial states psi0[b] (Sec. 4 starts every experiment from
    random states).  Per sample b, the final state is the dense circuit product
    applied to psi0[b] (so the per-sample offset, the interleaving of real and
    imaginary parts and the absence of a conjugate are all fixed), the
    expectations of the forward and of the backward are <psi|O|psi> of that
    state, and the backward gradients equal the parameter shift of expectations
    formed from dense products from the same psi0[b]."""
    rng = np.random.default_rng(11)
    for n in (2, 3, 5):
        gates = hea_gates(n, 2, ("RX", "RY", "RZ"), encoding=True, ring=n > 2)
        P = 2 * 3 * n
        theta = rng.uniform(0, 2 * math.pi, size=P)
        B = 3
        x = rng.uniform(-math.pi, math.pi, size=(B, n))
        psi0 = _random_states(rng, B, n)
        spec = ("IXYZ" * 2)[:n]
        xm, zm = pauli_string(spec)
        xms, zms = np.array([xm, 0], np.uint64), np.array([zm, 1], np.uint64)
        dense_obs = [_pauli_dense(spec), _pauli_dense("I" * (n - 1) + "Z")]
        E, psi = orc.forward(n, gates, theta, x, xms, zms, psi0=psi0, return_state=True)

        def dense_E(th, xb, p0):
            v = dense_state(n, gates, th, xb, psi0=p0)
            return np.array([np.vdot(v, O @ v).real for O in dense_obs])

        for b in range(B):
            ref = dense_state(n, gates, theta, x[b], psi0=psi0[b])
            np.testing.assert_allclose(psi[b], ref, atol=1e-12)
            np.testing.assert_allclose(E[b], dense_E(theta, x[b], psi0[b]), atol=1e-12)
        g = rng.normal(size=(B, 2))
        E1, dth, dx = orc.backward(n, gates, theta, x, xms, zms, g, psi0=psi0)
        np.testing.assert_allclose(E1, E, atol=1e-12)
        for p in range(0, P, 3):
            tp, tm = theta.copy(), theta.copy()
            tp[p] += math.pi / 2
            tm[p] -= math.pi / 2
            ref = sum(0.5 * float(g[b] @ (dense_E(tp, x[b], psi0[b]) - dense_E(tm, x[b], psi0[b])))
                      for b in range(B))
            np.testing.assert_allclose(dth[p], ref, atol=1e-11)
        for b in range(B):
            for f in range(n):
                xp, xn = x[b].copy(), x[b].copy()
                xp[f] += math.pi / 2
                xn[f] -= math.pi / 2
                ref = 0.5 * float(g[b] @ (dense_E(theta, xp, psi0[b]) - dense_E(theta, xn, psi0[b])))
                np.testing.assert_allclose(dx[b, f], ref, atol=1e-11)


ALL_PINS = [pin_p1_single_qubit, pin_p2_two_qubit, pin_p3_zero_angles, pin_p4_norm,
            pin_p5_dense, pin_p6_parameter_shift, pin_p7_backward_modes, pin_p9_pauli_expectation,
            pin_p10_cnot, pin_p11_initial_states]


# ---------------------------------------------------------------- loss helper (L1)
def pin_l1_losses(loss_and_grad_E):
    """The loss readings of the benchmarks against closed forms and invariants, not
    against a second copy of their formulas:
      * sum:      L = sum of all E; dL/dE = 1.
      * mean_sum: L = sum_b mean_k E; dL/dE = 1/K.
      * ce:       equal logits give L = log K and dL/dE = (1/K - [k = y]) / B;
                  with two classes the cross-entropy is the logistic loss
                  log(1 + exp(E_other - E_y)) (numpy's logaddexp), with gradient
                  -+sigmoid(E_other - E_y) / B; a constant added to one sample's
                  logits changes nothing; the batch loss is the mean of the
                  one-sample losses; every gradient row sums to 0; and dL/dE is
                  the central finite difference of L in every entry (which fixes
                  the 1/B of the mean)."""
    rng = np.random.default_rng(13)
    E = rng.normal(size=(5, 4))
    L, g = loss_and_grad_E(E, "sum")
    assert abs(L - E.sum()) <= 1e-12 and np.array_equal(g, np.ones_like(E))
    L, g = loss_and_grad_E(E, "mean_sum")
    assert abs(L - E.sum() / 4) <= 1e-12
    np.testing.assert_allclose(g, np.full_like(E, 0.25), atol=0)
    for K, B in ((3, 1), (10, 4)):
        lab = rng.integers(0, K, size=B)
        L, g = loss_and_grad_E(np.full((B, K), 0.37), "ce", lab)
        assert abs(L - math.log(K)) <= 1e-12
        ref = np.full((B, K), 1.0 / K)
        ref[np.arange(B), lab] -= 1.0
        np.testing.assert_allclose(g, ref / B, atol=1e-14)
    B = 6
    E2 = rng.normal(size=(B, 2)) * 2
    lab = rng.integers(0, 2, size=B)
    d = E2[np.arange(B), 1 - lab] - E2[np.arange(B), lab]
    L, g = loss_and_grad_E(E2, "ce", lab)
    assert abs(L - np.logaddexp(0.0, d).mean()) <= 1e-12
    sig = 1.0 / (1.0 + np.exp(-d))
    np.testing.assert_allclose(g[np.arange(B), lab], -sig / B, atol=1e-14)
    np.testing.assert_allclose(g[np.arange(B), 1 - lab], sig / B, atol=1e-14)
    K, B = 10, 7
    E3 = rng.normal(size=(B, K))
    lab = rng.integers(0, K, size=B)
    L, g = loss_and_grad_E(E3, "ce", lab)
    shift = E3 + rng.normal(size=(B, 1)) * 5
    L2, g2 = loss_and_grad_E(shift, "ce", lab)
    assert abs(L - L2) <= 1e-12
    np.testing.assert_allclose(g, g2, atol=1e-14)
    singles = [loss_and_grad_E(E3[b:b + 1], "ce", lab[b:b + 1])[0] for b in range(B)]
    assert abs(L - float(np.mean(singles))) <= 1e-12
    np.testing.assert_allclose(g.sum(axis=1), 0.0, atol=1e-15)
    h = 1e-6
    for b in range(B):
        for k in range(K):
            Ep, Em = E3.copy(), E3.copy()
            Ep[b, k] += h
            Em[b, k] -= h
            fd = (loss_and_grad_E(Ep, "ce", lab)[0] - loss_and_grad_E(Em, "ce", lab)[0]) / (2 * h)
            assert abs(g[b, k] - fd) <= 1e-8


LOSS_PINS = [pin_l1_losses]
