"""Planted mistakes in the relative-binning and calibration oracles must be caught by their pins.

Each case rebuilds the oracle module from its source with one plausible error and checks that at
least one pin of test_rb_oracle / test_cal_oracle fails. CPU only."""
import inspect
import sys
import types

import pytest

from oracle import cal_oracle, rb_oracle
from tests import test_cal_oracle as cal_pins
from tests import test_rb_oracle as rb_pins

RB_MUTATIONS = {
    "bound exponent sign": ("out += math.copysign(1.0, g) * (f / fg) ** g", "out += (f / fg) ** g"),
    "falling flank reversed": ("w[e, m] = (fe[e + 1] - f[m]) / (fe[e + 1] - fe[e])",
                               "w[e, m] = (f[m] - fe[e]) / (fe[e + 1] - fe[e])"),
    "summary without conj": ("c = 4.0 * df * np.conj(data) * h0 / psd", "c = 4.0 * df * data * h0 / psd"),
    "ratio inverted": ("r = he / h0e[i]", "r = h0e[i] / he"),
    "last edge dropped": ("if idx[-1] != len(f) - 1:\n        idx.append(len(f) - 1)", "pass"),
}
CAL_MUTATIONS = {
    "ghost node constant": ("ext = torch.cat([(2 * values[0] - values[1])[None], values, (2 * values[-1] - values[-2])[None]])",
                            "ext = torch.cat([values[0][None], values, values[-1][None]])"),
    "cubic coefficient": ("(3 * p0 - pm - 3 * p1 + p2) * t ** 3", "(3 * p0 - pm - 3 * p1 - p2) * t ** 3"),
    "phase sign": ("torch.exp(1j * dp.to(o.CDT))", "torch.exp(-1j * dp.to(o.CDT))"),
    "amplitude not offset": ("(1.0 + da).to(o.CDT)", "(da).to(o.CDT)"),
    "detector parameter block": ("base = 11 + 2 * nnode * i", "base = 11 + nnode * i"),
}


def _mutant(mod, old, new):
    src = inspect.getsource(mod)
    assert src.count(old) == 1, old
    m = types.ModuleType(mod.__name__ + "_mutant")
    m.__dict__["__name__"] = mod.__name__ + "_mutant"
    exec(compile(src.replace(old, new), mod.__name__ + "_mutant", "exec"), m.__dict__)
    return m


def _caught(pins, fixture_name):
    fns = [getattr(pins, n) for n in dir(pins) if n.startswith("test_")]
    fx = getattr(pins, fixture_name).__wrapped__() if hasattr(getattr(pins, fixture_name), "__wrapped__") else None
    failed = []
    for fn in fns:
        try:
            params = inspect.signature(fn).parameters
            fn(*([fx] if params else []))
        except Exception:
            failed.append(fn.__name__)
    return failed


@pytest.mark.parametrize("name", sorted(RB_MUTATIONS))
def test_rb_mutation_is_caught(name, monkeypatch):
    monkeypatch.setattr(rb_pins, "rb", _mutant(rb_oracle, *RB_MUTATIONS[name]))
    assert _caught(rb_pins, "small"), f"no pin caught: {name}"


@pytest.mark.parametrize("name", sorted(CAL_MUTATIONS))
def test_cal_mutation_is_caught(name, monkeypatch):
    monkeypatch.setattr(cal_pins, "cal", _mutant(cal_oracle, *CAL_MUTATIONS[name]))
    assert _caught(cal_pins, "ev"), f"no pin caught: {name}"


def test_unmutated_oracles_pass_every_pin():
    """The harness itself: without a planted mistake no pin fails."""
    assert _caught(rb_pins, "small") == []
    assert _caught(cal_pins, "ev") == []
