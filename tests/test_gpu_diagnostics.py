"""Diagnostics of the library on the GPU: the microbenchmarks behind the
measured peaks the benchmark reports beside the published ones."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_plausible():
    # MI355X publishes 78.6 TFLOP/s for FP64 and non-packed FP32 vector FMA;
    # the microbenchmarks must land in a band around that (and LDS reads in
    # the tens of TB/s: 256 CUs x 128 B per clock at 2.4 GHz is 78.6 TB/s)
    import torch
    from paper_1303_6615_amd.binding import measure_peaks
    assert torch.cuda.is_available()
    p = measure_peaks()
    assert 20.0 < p["fp32_tflops"] < 200.0, p
    assert 10.0 < p["fp64_tflops"] < 120.0, p
    assert 5.0 < p["lds_tbps"] < 200.0, p
