"""The measured roofline ceiling (lll_fp32_fma_peak): plain FP32 FMAs reach a
large part of, and never exceed, the single-issue rate implied by the quoted
vector peak (157.3 TFLOP/s counts dual-issue packed FMAs; half of it is the
rate of one FMA per lane and cycle)."""
import pytest

pytestmark = pytest.mark.gpu


def test_fma_probe_is_below_the_single_issue_rate(gpu_lib):
    t = gpu_lib.fp32_fma_peak()
    print(f"plain FP32 FMA throughput {t:.1f} TFLOP/s")
    assert 40.0 < t <= 157.3 / 2 * 1.02
