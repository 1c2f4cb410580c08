"""Plausible slips planted in a copy of the display oracle must each fail a pin.

The mutated copy is loaded as a module of the ``oracle`` package (so its relative imports
resolve) and swapped in for ``oracle.display`` while the pins of
test_oracle_display_pins.py run.
"""
import importlib.util
import os

import pytest

import oracle
import test_oracle_display_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "display.py")

MUTATIONS = [
    ("ratio not normalised", "np.clip(a[c] / am[c], 0.0, 1.0)", "np.clip(a[c], 0.0, 1.0)"),
    ("interlace swapped", "np.where(even[None], pm, pp)", "np.where(even[None], pp, pm)"),
    ("field phase dropped", "return phi - theta, phi + theta", "return -theta, theta"),
    ("arcsin for arccos", "theta = np.arccos(r)", "theta = np.arcsin(r)"),
    ("filter a full band wide", "mx = np.abs(signed_freq_index(grid.nx)) * 4 < grid.nx",
     "mx = np.abs(signed_freq_index(grid.nx)) * 2 < grid.nx"),
    ("propagation sign", "transfer(grid, lam, d) * mask", "transfer(grid, lam, -d) * mask"),
    ("intensity not squared", "else np.abs(st) ** 2", "else np.abs(st)"),
    ("phase input as a real field", "np.exp(1j * np.asarray(inp, dtype=np.float64))",
     "np.cos(np.asarray(inp, dtype=np.float64)).astype(np.complex128)"),
]

PINS = [getattr(pins, n) for n in dir(pins) if n.startswith("test_")]


def load_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert old in src, old
    path = tmp_path / "display_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle.display_mutant", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(tmp_path, monkeypatch, name, old, new):
    mod = load_mutant(tmp_path, old, new)
    monkeypatch.setattr(pins, "dp", mod)
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, "mutation '%s' passed every pin" % name
