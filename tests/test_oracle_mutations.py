"""The oracle's pins are sensitive: planting a plausible mistake in a copy of the C
oracle (on the CPU) makes at least one pin fail.  Each mutation below is a slip a
reader could make when transcribing Eq. 4, 10 or 12 or their derivatives."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gws_oracle.c")

PH = ("const double ph = phase[i] - TWO_PI * (gx * mean_x[i] + gy * mean_y[i])\n"
      "                                    + TWO_PI * (-depth[i]) * kz;\n                    re")
QUAD = ("const double quad = gx * gx * cov_xx[i] + 2.0 * gx * gy * cov_xy[i]\n"
        "                                      + gy * gy * cov_yy[i];\n                    const double mag")
SHIFT = "const double gx = nu_x - ref_nu_x, gy = nu_y - ref_nu_y;   /* argument of g_i */"
MUTATIONS = {
    "ramp_sign": (PH, PH.replace("phase[i] - TWO_PI", "phase[i] + TWO_PI")),
    "propagation_sign": (PH, PH.replace("(-depth[i])", "(depth[i])")),
    "dropped_phase": (PH, PH.replace("phase[i] - TWO_PI", "- TWO_PI")),
    "det_instead_of_sqrt": ("* TWO_PI * sqrt(det) * exp", "* TWO_PI * det * exp"),
    "dropped_2pi": ("* TWO_PI * sqrt(det) * exp", "* sqrt(det) * exp"),
    "envelope_pi2": ("sqrt(det) * exp(-2.0 * PI * PI * quad);\n                    /* phase",
                     "sqrt(det) * exp(-1.0 * PI * PI * quad);\n                    /* phase"),
    "transposed_cov": (QUAD, QUAD.replace("gx * gx * cov_xx[i]", "gx * gx * cov_yy[i]")
                       .replace("gy * gy * cov_yy[i]", "gy * gy * cov_xx[i]")),
    "cross_term_sign": (QUAD, QUAD.replace("+ 2.0 * gx", "- 2.0 * gx")),
    "no_evanescent_cut": ("if (nu2 < inv_l * inv_l) {", "if (1) {"),
    "pitch_axis": ("signed_index(freq_my[f], ny) / (ny * py)", "signed_index(freq_my[f], ny) / (ny * px)"),
    "grad_phase_sign": ("g_phi += RE_CONJ_Q(-t_im, t_re);", "g_phi += RE_CONJ_Q(t_im, -t_re);"),
    "grad_cov_xy_factor": ("- 4.0 * PI * PI * gx * gy;", "- 2.0 * PI * PI * gx * gy;"),
    "grad_mean_axis": ("g_mx += RE_CONJ_Q(TWO_PI * gx * t_im, -TWO_PI * gx * t_re);",
                       "g_mx += RE_CONJ_Q(TWO_PI * gy * t_im, -TWO_PI * gy * t_re);"),
    "grad_opacity": ("g_o += amp[(int64_t)c * n + i] * RE_CONJ_Q(b_re, b_im);",
                     "g_o += RE_CONJ_Q(b_re, b_im);"),
    # reference plane wave (Sec. 4.1): shift sign, shift left out of the ramp, shift also
    # applied to the transfer function, shift dropped from the gradient's frequency weights
    "ref_shift_sign": (SHIFT, SHIFT.replace("nu_x - ref_nu_x", "nu_x + ref_nu_x")),
    "ref_ramp_unshifted": (PH, PH.replace("(gx * mean_x[i] + gy * mean_y[i])", "(nu_x * mean_x[i] + nu_y * mean_y[i])")),
    "ref_shift_in_transfer": ("        const double nu2 = nu_x * nu_x + nu_y * nu_y;\n        const double gx",
                              "        const double nu2 = (nu_x - ref_nu_x) * (nu_x - ref_nu_x)"
                              " + (nu_y - ref_nu_y) * (nu_y - ref_nu_y);\n        const double gx"),
    "ref_grad_unshifted": ("const double gx = nu_x - ref_nu_x, gy = nu_y - ref_nu_y;\n                    const double quad",
                           "const double gx = nu_x, gy = nu_y;\n                    const double quad"),
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
