"""Planted mistakes in the nested-sampling oracle must be caught by its pins.

Each case rebuilds the oracle module from its source with one plausible error (a wrong order,
an off-by-one in a volume decrement, a strict inequality, a sign) and checks that at least one
pin in test_ns_oracle fails. The mistakes exist only inside this CPU test.
"""
import importlib.util
import inspect
import types

import pytest

from oracle import ns_oracle
from tests import test_ns_oracle as pins

MUTATIONS = {
    "descending order": ('ok = ok[np.argsort(cl[ok], kind="stable")]',
                         'ok = ok[np.argsort(-cl[ok], kind="stable")]'),
    "order decrement off by one": ("d = 1.0 / (K + nacc - j + 1)", "d = 1.0 / (K + nacc - j)"),
    "no special first decrement": ('if volume == "paper" or j == 1:', 'if volume == "paper":'),
    "strict acceptance": ("ok = np.where(cl >= l_min)[0]", "ok = np.where(cl > l_min)[0]"),
    "dX from the new contour": ("ln_dx = ln_x + _log_one_minus_exp(d)", "ln_dx = ln_x - d + _log_one_minus_exp(d)"),
    "final shares of all volume": ("ln_share = ln_x - math.log(K)", "ln_share = -math.log(K)"),
    "stop on the live minimum": ("bound = _logaddexp(ln_z, float(np.max(live_l)) + ln_x)",
                                 "bound = _logaddexp(ln_z, float(np.min(live_l)) + ln_x)"),
}

PINS = [pins.test_serial_case_volume_is_minus_i_over_k, pins.test_tiny_run_by_hand,
        pins.test_constant_likelihood_gives_its_value, pins.test_paper_volume_is_biased_when_many_replace_at_once,
        pins.test_gaussian_evidence_and_posterior_moments, pins.test_invariants_with_prior_draws]


def _mutant(old, new):
    src = inspect.getsource(ns_oracle)
    assert src.count(old) == 1, old
    mod = types.ModuleType("ns_oracle_mutant")
    exec(compile(src.replace(old, new), "ns_oracle_mutant", "exec"), mod.__dict__)
    return mod


def _fails(fn):
    try:
        if "n" in inspect.signature(fn).parameters:
            for n in (1, 16, 400):
                fn(n)
        else:
            fn()
    except (AssertionError, ValueError, FloatingPointError, ZeroDivisionError, IndexError):
        return True
    return False


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    monkeypatch.setattr(pins, "ns", _mutant(*MUTATIONS[name]))
    caught = [f.__name__ for f in PINS + [pins.test_contour_volumes_match_the_ball] if _fails(f)]
    assert caught, f"no pin caught: {name}"
