"""The FMA probe that places the published vector-ALU peaks on the device."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_peak_reports_the_device(gpu):
    from paper_2609_29253_amd import _lib
    pk = _lib.probe_peak(0)
    print(f"FMA probe: {pk}", flush=True)
    assert pk["compute_units"] > 0 and pk["clock_ghz"] > 0
    # below the published 78.6 TFLOP/s per precision (with packed FP32 off) and
    # far above what a broken timing would give
    for key in ("fp64_flops", "fp32_flops"):
        assert 1e12 < pk[key] < 1.2 * 2 * 64 * pk["compute_units"] * pk["clock_ghz"] * 1e9
