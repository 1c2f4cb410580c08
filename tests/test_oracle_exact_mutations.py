"""Plausible slips planted in a copy of the exact-blending oracle must each fail a pin.

The mutated copy is loaded as a module of the ``oracle`` package (so its relative imports
resolve) and swapped in for ``oracle.exact`` while the pins of test_oracle_exact_pins.py run.
"""
import importlib.util
import os

import pytest

import oracle
import test_oracle_exact_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "exact.py")

MUTATIONS = [
    ("back to front", "order = depth_order(scene)", "order = depth_order(scene)[::-1]"),
    ("no alpha threshold", "alpha = np.where(alpha > t_eps, alpha, 0.0)", "alpha = alpha + 0.0"),
    ("mask ignored", "S = spectrum_from_field_fft(T * u, grid)", "S = spectrum_from_field_fft(u, grid)"),
    ("self-occlusion", "S = spectrum_from_field_fft(T * u, grid)",
     "S = spectrum_from_field_fft(T * (1.0 - float(scene.opacity[k]) * np.abs(u)) * u, grid)"),
    ("alpha without opacity", "alpha = o * np.abs(u)", "alpha = np.abs(u)"),
    ("propagation sign", "transfer(grid, grid.lambdas[c], -z)", "transfer(grid, grid.lambdas[c], z)"),
    ("no opacity in the splat", "U[c] += a * o * transfer", "U[c] += a * transfer"),
    ("centring dropped", "np.fft.fft2(u, axes=(-2, -1)) * fy[:, None] * fx[None, :]",
     "np.fft.fft2(u, axes=(-2, -1))"),
    ("phase dropped", "return field_from_spectrum_fft(spectrum(one, g1, ordered=False)[0], grid)",
     "return np.abs(field_from_spectrum_fft(spectrum(one, g1, ordered=False)[0], grid))"),
]

PINS = [getattr(pins, n) for n in dir(pins) if n.startswith("test_")]


def load_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert old in src, old
    path = tmp_path / "exact_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle.exact_mutant", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(tmp_path, monkeypatch, name, old, new):
    mod = load_mutant(tmp_path, old, new)
    monkeypatch.setattr(pins, "ex", mod)
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, "mutation '%s' passed every pin" % name
