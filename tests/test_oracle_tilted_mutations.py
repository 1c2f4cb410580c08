"""Plausible slips planted in a copy of the tilted-Gaussian oracle must each fail a pin.

The mutated copy is loaded as a module of the ``oracle`` package and swapped in for
``oracle.tilted`` while the pins of test_oracle_tilted_pins.py run.
"""
import importlib.util
import os

import pytest

import oracle
import test_oracle_tilted_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "tilted.py")

MUTATIONS = [
    ("rotation not transposed (R k instead of R^T k)",
     "kox = R[0, 0] * nux + R[1, 0] * nuy + R[2, 0] * kz", "kox = R[0, 0] * nux + R[0, 1] * nuy + R[0, 2] * kz"),
    ("det J dropped", "detj = np.abs(koz) / kz", "detj = 1.0 + 0.0 * koz"),
    ("det J inverted", "detj = np.abs(koz) / kz", "detj = kz / np.abs(koz)"),
    ("det J signed", "detj = np.abs(koz) / kz", "detj = koz / kz"),
    ("det J from the wrong column", "koz = R[0, 2] * nux + R[1, 2] * nuy + R[2, 2] * kz",
     "koz = R[2, 0] * nux + R[2, 1] * nuy + R[2, 2] * kz"),
    ("scales swapped", "(su * su * kox * kox + sv * sv * koy * koy)", "(sv * sv * kox * kox + su * su * koy * koy)"),
    ("exponent pi^2 instead of 2 pi^2", "np.exp(-2.0 * math.pi ** 2 * (su", "np.exp(-math.pi ** 2 * (su"),
    ("det S dropped", "2.0 * math.pi * su * sv * np.exp", "2.0 * math.pi * np.exp"),
    ("ramp sign", "ramp = np.exp(-2j * math.pi", "ramp = np.exp(2j * math.pi"),
    ("propagation sign", "np.exp(2j * math.pi * (-z) * kz)", "np.exp(2j * math.pi * z * kz)"),
    ("k_z of the first wavelength only", "gaussian_spectrum(R, su, sv, nux, nuy, lam)",
     "gaussian_spectrum(R, su, sv, nux, nuy, grid.lambdas[0])"),
    ("k_z without the transverse part", "w2 = inv_l * inv_l - (nux * nux + nuy * nuy)", "w2 = inv_l * inv_l + 0.0 * nux"),
]

PINS = [getattr(pins, n) for n in dir(pins) if n.startswith("test_")]


def load_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert old in src, old
    path = tmp_path / "tilted_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle.tilted_mutant", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def run_pins():
    failed = []
    for pin in PINS:
        args = [(0,), (1,)] if pin.__name__ == "test_field_matches_plane_wave_superposition" else [()]
        for a in args:
            try:
                pin(*a)
            except Exception:           # an assertion, or a slip that breaks the arithmetic outright
                failed.append(pin.__name__)
    return failed


def test_unmutated_oracle_passes_every_pin():
    assert run_pins() == []


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(tmp_path, monkeypatch, name, old, new):
    mod = load_mutant(tmp_path, old, new)
    monkeypatch.setattr(pins, "tl", mod)
    assert run_pins(), "mutation '%s' passed every pin" % name
