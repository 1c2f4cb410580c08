"""The oracle's pins are sensitive: planting a plausible mistake in a copy of the C
oracle (on the CPU) makes at least one pin fail.  Each mutation below is a slip a
reader could make when transcribing Eq. 4, 10 or 12 or their derivatives."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gws_oracle.c")

PH = ("const double ph = phase[i] - TWO_PI * (nu_x * mean_x[i] + nu_y * mean_y[i])\n"
      "                                    + TWO_PI * (-depth[i]) * kz;\n                    re")
QUAD = ("const double quad = nu_x * nu_x * cov_xx[i] + 2.0 * nu_x * nu_y * cov_xy[i]\n"
        "                                      + nu_y * nu_y * cov_yy[i];\n                    const double mag")
MUTATIONS = {
    "ramp_sign": (PH, PH.replace("phase[i] - TWO_PI", "phase[i] + TWO_PI")),
    "propagation_sign": (PH, PH.replace("(-depth[i])", "(depth[i])")),
    "dropped_phase": (PH, PH.replace("phase[i] - TWO_PI", "- TWO_PI")),
    "det_instead_of_sqrt": ("* TWO_PI * sqrt(det) * exp", "* TWO_PI * det * exp"),
    "dropped_2pi": ("* TWO_PI * sqrt(det) * exp", "* sqrt(det) * exp"),
    "envelope_pi2": ("sqrt(det) * exp(-2.0 * PI * PI * quad);\n                    /* phase",
                     "sqrt(det) * exp(-1.0 * PI * PI * quad);\n                    /* phase"),
    "transposed_cov": (QUAD, QUAD.replace("nu_x * nu_x * cov_xx[i]", "nu_x * nu_x * cov_yy[i]")
                       .replace("nu_y * nu_y * cov_yy[i]", "nu_y * nu_y * cov_xx[i]")),
    "cross_term_sign": (QUAD, QUAD.replace("+ 2.0 * nu_x", "- 2.0 * nu_x")),
    "no_evanescent_cut": ("if (nu2 < inv_l * inv_l) {", "if (1) {"),
    "pitch_axis": ("signed_index(freq_my[f], ny) / (ny * py)", "signed_index(freq_my[f], ny) / (ny * px)"),
    "grad_phase_sign": ("g_phi += RE_CONJ_Q(-t_im, t_re);", "g_phi += RE_CONJ_Q(t_im, -t_re);"),
    "grad_cov_xy_factor": ("- 4.0 * PI * PI * nu_x * nu_y;", "- 2.0 * PI * PI * nu_x * nu_y;"),
    "grad_mean_axis": ("g_mx += RE_CONJ_Q(TWO_PI * nu_x * t_im, -TWO_PI * nu_x * t_re);",
                       "g_mx += RE_CONJ_Q(TWO_PI * nu_y * t_im, -TWO_PI * nu_y * t_re);"),
    "grad_opacity": ("g_o += amp[(int64_t)c * n + i] * RE_CONJ_Q(b_re, b_im);",
                     "g_o += RE_CONJ_Q(b_re, b_im);"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(SRC).read()
    before, after = MUTATIONS[name]
    assert src.count(before) == 1, name
    path = tmp_path / ("mut_%s.c" % name)
    path.write_text(src.replace(before, after))
    env = dict(os.environ, GWS_ORACLE_SRC=str(path))
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-q", "-x", "-p", "no:cacheprovider"], env=env, capture_output=True, text=True, cwd=ROOT)
    assert r.returncode != 0, "planted mistake %s passed every pin:\n%s" % (name, r.stdout[-2000:])
