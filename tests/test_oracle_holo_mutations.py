"""Plausible slips planted in a copy of the holographics oracle must each fail a pin.

The mutated copy is loaded as a module of the ``oracle`` package and swapped in for
``oracle.holographics`` while the pins of test_oracle_holo_pins.py run.
"""
import importlib.util
import os

import pytest

import oracle
import test_oracle_holo_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "holographics.py")

MUTATIONS = [
    ("Jacobian depth column sign", 'cam["fx"] * p[0] * iz * iz', '-cam["fx"] * p[0] * iz * iz'),
    ("view translation dropped", "p = Rv @ mu_w + t", "p = Rv @ mu_w"),
    ("view rotation transposed", "Sigma_r = J @ Rv @ Sigma_w @ Rv.T @ J.T", "Sigma_r = J @ Rv.T @ Sigma_w @ Rv @ J.T"),
    ("view direction reversed", "real_sh(deg, mu_w - centre)", "real_sh(deg, centre - mu_w)"),
    ("quaternion read as (x, y, z, w)", "w, x, y, z = np.asarray(q", "x, y, z, w = np.asarray(q"),
    ("scales squared", "np.diag(np.asarray(scale, dtype=np.float64))", "np.diag(np.asarray(scale, dtype=np.float64) ** 2)"),
    ("depth map ignored", '[0.0, 0.0, cam["depth_scale"]]', "[0.0, 0.0, 1.0]"),
    ("opacity not clamped", "opacity=min(max(o, 0.0), 1.0)", "opacity=o"),
    ("real part for m < 0", "math.sqrt(2.0) * y.imag if m < 0", "math.sqrt(2.0) * y.real if m < 0"),
]

PINS = [getattr(pins, n) for n in dir(pins) if n.startswith("test_")]


def load_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert old in src, old
    path = tmp_path / "holographics_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle.holographics_mutant", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(tmp_path, monkeypatch, name, old, new):
    mod = load_mutant(tmp_path, old, new)
    monkeypatch.setattr(pins, "hg", mod)
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
        except Exception:           # a slip that breaks the arithmetic outright also counts
            failed.append(pin.__name__)
    assert failed, "mutation '%s' passed every pin" % name
