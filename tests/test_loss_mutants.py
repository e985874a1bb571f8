"""Every plausible mistake planted in the oracle's loss helper is caught by a pin.

Each mutant is a copy of ``oracle/oracle.py`` with one textual substitution in
``loss_and_grad_E`` (a dropped 1/B, a sum for a mean, a softmax over the wrong
axis, a wrong sign ...), loaded as a fresh module.  The loss pins of
``oracle_pins`` must reject every mutant, and pass on the unmodified helper.
"""
import importlib.util

import pytest

import oracle_pins
from oracle import oracle as oracle_mod

MUTANTS = [
    ("ce_grad_without_batch_mean", "return L, g / B", "return L, g"),
    ("ce_loss_sum_not_mean", "L = float(-np.log(p[np.arange(B), lab]).mean())",
     "L = float(-np.log(p[np.arange(B), lab]).sum())"),
    ("ce_label_added_not_subtracted", "g[np.arange(B), lab] -= 1.0", "g[np.arange(B), lab] += 1.0"),
    ("ce_softmax_over_batch", "p = ex / ex.sum(axis=1, keepdims=True)", "p = ex / ex.sum(axis=0, keepdims=True)"),
    ("ce_shift_per_class", "m = E.max(axis=1, keepdims=True)", "m = E.max(axis=0, keepdims=True)"),
    ("ce_loss_of_wrong_class", "L = float(-np.log(p[np.arange(B), lab]).mean())",
     "L = float(-np.log(p[np.arange(B), (lab + 1) % K]).mean())"),
    ("ce_no_log", "L = float(-np.log(p[np.arange(B), lab]).mean())",
     "L = float(-(p[np.arange(B), lab]).mean())"),
    ("mean_sum_divides_by_batch", "return float(E.mean(axis=1).sum()), np.full_like(E, 1.0 / K)",
     "return float(E.mean(axis=1).sum()), np.full_like(E, 1.0 / B)"),
    ("mean_sum_loss_over_batch", "return float(E.mean(axis=1).sum())", "return float(E.mean(axis=0).sum())"),
    ("sum_grad_halved", "return float(E.sum()), np.ones_like(E)", "return float(E.sum()), 0.5 * np.ones_like(E)"),
]


def _load(src, name, tmp_path):
    path = tmp_path / f"oracle_{name}.py"
    path.write_text(src)
    spec = importlib.util.spec_from_file_location(f"oracle_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.loss_and_grad_E


def test_loss_pins_pass():
    for pin in oracle_pins.LOSS_PINS:
        pin(oracle_mod.loss_and_grad_E)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_loss_mutant_is_caught(name, old, new, tmp_path):
    src = open(oracle_mod.__file__).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    fn = _load(src.replace(old, new), name, tmp_path)
    caught = []
    for pin in oracle_pins.LOSS_PINS:
        try:
            pin(fn)
        except (AssertionError, ValueError, IndexError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} survives every loss pin"
