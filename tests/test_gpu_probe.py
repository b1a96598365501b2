"""The FMA probe that places the published vector-ALU peaks on the device."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_peak_reports_the_device(gpu):
    from paper_2609_29253_amd import _lib
    pk = _lib.probe_peak(0)
    print(f"FMA probe: {pk}", flush=True)
    assert pk["compute_units"] > 0 and pk["clock_ghz"] > 0
    # below the published peaks with a margin for clock boost (FP64: 64 FMA
    # lanes per CU and clock, 78.6 TFLOP/s; FP32: 128, 157.3 TFLOP/s, of which
    # unpacked FMA reaches about two thirds) and far above what a broken timing
    # would give
    for key, lanes in (("fp64_flops", 64), ("fp32_flops", 128)):
        assert 1e12 < pk[key] < 1.2 * 2 * lanes * pk["compute_units"] * pk["clock_ghz"] * 1e9
