"""Every plausible mistake planted in the oracle is caught by at least one pin.

Each mutant is a copy of ``oracle/qfo.c`` with one textual substitution (a wrong
sign, a dropped factor, a transposed operand, a wrong bit index ...), compiled
to a temporary library.  The pins of ``oracle_pins`` must reject every mutant;
a mutant that survives means the pins leave part of the oracle unchecked.
"""
import os
import subprocess
import tempfile

import pytest

import oracle_pins
from oracle.oracle import SRC_PATH, Oracle

# (name, original text, replacement, which occurrence: 0-based or None for all)
MUTANTS = [
    ("Y_transposed", "p.m[1] = c_make(0.0, -1.0);\n    p.m[2] = c_make(0.0, 1.0);",
     "p.m[1] = c_make(0.0, 1.0);\n    p.m[2] = c_make(0.0, -1.0);", None),
    ("rotation_sign", "u.m[i] = c_mul(c_make(0.0, -s), p.m[i]);",
     "u.m[i] = c_mul(c_make(0.0, s), p.m[i]);", None),
    ("full_angle_in_u", "double c = cos(0.5 * phi), s = sin(0.5 * phi);",
     "double c = cos(phi), s = sin(phi);", 0),
    ("full_angle_in_du", "double c = cos(0.5 * phi), s = sin(0.5 * phi);",
     "double c = cos(phi), s = sin(phi);", 1),
    ("du_dropped_half", "c_make(0.0, -0.5 * c)", "c_make(0.0, -1.0 * c)", None),
    ("du_sin_sign", "c_make(-0.5 * s, 0.0)", "c_make(0.5 * s, 0.0)", None),
    ("dagger_without_transpose", "d.m[1] = c_conj(u.m[2]);\n  d.m[2] = c_conj(u.m[1]);",
     "d.m[1] = c_conj(u.m[1]);\n  d.m[2] = c_conj(u.m[2]);", None),
    ("dagger_without_conj", "d.m[0] = c_conj(u.m[0]);", "d.m[0] = u.m[0];", None),
    ("pair_update_transposed", "psi[i] = c_add(c_mul(u.m[0], a0), c_mul(u.m[1], a1));\n"
     "    psi[i | step] = c_add(c_mul(u.m[2], a0), c_mul(u.m[3], a1));",
     "psi[i] = c_add(c_mul(u.m[0], a0), c_mul(u.m[2], a1));\n"
     "    psi[i | step] = c_add(c_mul(u.m[1], a0), c_mul(u.m[3], a1));", None),
    ("big_endian_target", "step = (int64_t)1 << t, i;\n#pragma omp parallel for schedule(static) if (n >= 16)\n"
     "  for (i = 0; i < dim; ++i) {\n    if (i & step) continue;\n    cplx a0 = psi[i], a1 = psi[i | step];\n"
     "    psi[i] =",
     "step = (int64_t)1 << (n - 1 - t), i;\n#pragma omp parallel for schedule(static) if (n >= 16)\n"
     "  for (i = 0; i < dim; ++i) {\n    if (i & step) continue;\n    cplx a0 = psi[i], a1 = psi[i | step];\n"
     "    psi[i] =", None),
    ("cz_or_instead_of_and", "if ((i & mc) && (i & mt))", "if ((i & mc) || (i & mt))", None),
    ("seed_without_factor_2", "c_scale(tmp[i], 2.0 * g)", "c_scale(tmp[i], g)", None),
    ("grad_without_conj", "acc += c_mul(c_conj(lam[i]), k0).re + c_mul(c_conj(lam[i | step]), k1).re;",
     "acc += c_mul(lam[i], k0).re + c_mul(lam[i | step], k1).re;", None),
    ("grad_uses_u_not_du", "gr = grad_term(lam, prev, n, g[1], drot(g[0], phi));",
     "gr = grad_term(lam, prev, n, g[1], rot(g[0], phi));", None),
    ("psi_unapply_with_u", "apply_1q(psi, n, g[1], dagger(u));    /* psi <- psi_{j-1} */",
     "apply_1q(psi, n, g[1], u);    /* psi <- psi_{j-1} */", None),
    ("lambda_update_with_u", "apply_1q(lam, n, g[1], dagger(u));       /* lambda <- lambda_{j-1} */",
     "apply_1q(lam, n, g[1], u);       /* lambda <- lambda_{j-1} */", None),
    ("grad_after_lambda_update",
     "gr = grad_term(lam, prev, n, g[1], drot(g[0], phi));\n"
     "        if (g[3] >= 0) gth[(int64_t)b * n_params + g[3]] += gr;\n"
     "        else if (dx) dx[(int64_t)b * n_inputs + g[4]] += gr;\n"
     "        apply_1q(lam, n, g[1], dagger(u));       /* lambda <- lambda_{j-1} */",
     "apply_1q(lam, n, g[1], dagger(u));       /* lambda <- lambda_{j-1} */\n"
     "        gr = grad_term(lam, prev, n, g[1], drot(g[0], phi));\n"
     "        if (g[3] >= 0) gth[(int64_t)b * n_params + g[3]] += gr;\n"
     "        else if (dx) dx[(int64_t)b * n_inputs + g[4]] += gr;", None),
    ("lambda_skips_cz", "        apply_cz(lam, n, g[1], g[2]);\n", "", None),
    ("pauli_sign_before_flip", "popcount64(src & zm)", "popcount64((uint64_t)i & zm)", None),
    ("pauli_no_y_phase", "int ny = popcount64(xm & zm) & 3;", "int ny = 0;", None),
    ("theta_grad_overwritten", "gth[(int64_t)b * n_params + g[3]] += gr;",
     "gth[(int64_t)b * n_params + g[3]] = gr;", None),
    ("input_grad_overwritten", "dx[(int64_t)b * n_inputs + g[4]] += gr;",
     "dx[(int64_t)b * n_inputs + g[4]] = gr;", None),
    ("input_angle_from_theta", "return g[3] >= 0 ? theta[g[3]] : xb[g[4]];",
     "return g[3] >= 0 ? theta[g[3]] : theta[g[4]];", None),
    ("cnot_on_control_clear", "if ((i & mc) && !(i & mt)) {", "if (!(i & mc) && !(i & mt)) {", None),
    ("cnot_control_target_swapped", "else if (g[0] == QFO_CNOT) apply_cnot(psi, n, g[1], g[2]);",
     "else if (g[0] == QFO_CNOT) apply_cnot(psi, n, g[2], g[1]);", None),
    ("lambda_skips_cnot", "        apply_cnot(lam, n, g[1], g[2]);\n", "", None),
    ("psi0_offset_forward", "init_state(psi, n, psi0 ? psi0 + 2 * dim * b : NULL);",
     "init_state(psi, n, psi0 ? psi0 + dim * b : NULL);", 0),
    ("psi0_offset_backward", "init_state(psi, n, psi0 ? psi0 + 2 * dim * b : NULL);",
     "init_state(psi, n, psi0 ? psi0 + dim * b : NULL);", 1),
    ("psi0_ignored_in_backward", "init_state(psi, n, psi0 ? psi0 + 2 * dim * b : NULL);",
     "init_state(psi, n, NULL);", 1),
    ("psi0_conjugated_load", "psi[i] = c_make(psi0_b[2 * i], psi0_b[2 * i + 1]);",
     "psi[i] = c_make(psi0_b[2 * i], -psi0_b[2 * i + 1]);", None),
    ("psi0_parts_swapped", "psi[i] = c_make(psi0_b[2 * i], psi0_b[2 * i + 1]);",
     "psi[i] = c_make(psi0_b[2 * i + 1], psi0_b[2 * i]);", None),
    ("batch_sum_first_sample_only", "for (b = 0; b < B; ++b) acc += gth[(int64_t)b * n_params + p];",
     "for (b = 0; b < 1; ++b) acc += gth[(int64_t)b * n_params + p];", None),
]


def _mutate(src, old, new, occ):
    assert old in src, f"mutation anchor not found: {old[:60]!r}"
    if occ is None:
        return src.replace(old, new)
    parts = src.split(old)
    assert len(parts) > occ + 1
    return old.join(parts[: occ + 1]) + new + old.join(parts[occ + 1:])


@pytest.mark.parametrize("name,old,new,occ", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, occ, tmp_path):
    src = open(SRC_PATH).read()
    mutated = _mutate(src, old, new, occ)
    assert mutated != src
    c = tmp_path / f"qfo_{name}.c"
    so = tmp_path / f"libqfo_{name}.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-std=c99", "-fopenmp", "-shared", "-fPIC", str(c), "-o", str(so), "-lm"],
                   check=True)
    orc = Oracle(str(so))
    caught = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} survives every pin"
