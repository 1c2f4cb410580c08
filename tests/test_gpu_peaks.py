"""Measured roofline denominators (gws_measure_peaks) are plausible for an MI355X."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_peaks_plausible():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    p = gws.context(0).measure_peaks()
    print(p, flush=True)
    # derived peaks: transcendentals 19.66e12 /s, FP32 VALU ops 78.6e12 /s, HBM 8e12 B/s
    assert 5e12 < p["trans_ops_per_s"] < 1.05 * 19.66e12
    assert 2e13 < p["valu_ops_per_s"] < 1.05 * 78.6e12
    assert 1e12 < p["hbm_bytes_per_s"] < 1.05 * 8e12
