"""The FP64 FMA calibration entry point on the GPU: a rate in the range the
hardware allows (above a quarter of the nominal 78.6 TFLOP/s, at most 5 %
above it, which would mean a clock above the nominal 2.4 GHz)."""

import pytest

pytestmark = pytest.mark.gpu


def test_fp64_fma_calibration_rate():
    from paper_2306_05002_amd import dg2p
    r = dg2p.calibrate_fp64_fma()
    print("fp64 vector FMA TFLOP/s", r)
    assert 0.25 * 78.6 < r <= 1.05 * 78.6
