"""The measured roofline ceilings: lll_fp32_fma_peak (independent FP32 FMA
chains whose multiplier and addend are kernel arguments, i.e. scalar-register
operands) and lll_fp32_mix_peak (the quadrature recursion's mix: per node and
rate two FMAs with a scalar-register table operand and one on vector registers
only).  Both stay below the quoted vector peak (157.3 TFLOP/s, which counts
packed FMAs); the scalar-operand probe stays near the one-FMA-per-lane-and-cycle
rate (78.65 TFLOP/s).  lll_fp32_mfma_peak: independent FP32 16x16x4
matrix-core instructions, the exact-drift kernel's ceiling."""
import pytest

pytestmark = pytest.mark.gpu


def test_fma_probe_is_below_the_single_issue_rate(gpu_lib):
    t = gpu_lib.fp32_fma_peak()
    print(f"plain FP32 FMA throughput {t:.1f} TFLOP/s")
    assert 40.0 < t <= 157.3 / 2 * 1.05


def test_mix_probe_is_below_the_quoted_peak(gpu_lib):
    t = gpu_lib.fp32_mix_peak()
    print(f"quadrature-recursion instruction mix {t:.1f} TFLOP/s")
    assert 40.0 < t <= 157.3


def test_mfma_probe_is_below_the_quoted_matrix_peak(gpu_lib):
    """The FP32 matrix-core ceiling used for the exact-drift kernel's
    roofline: a positive rate no higher than the quoted dense FP32 matrix
    peak (157.3 TFLOP/s)."""
    t = gpu_lib.fp32_mfma_peak()
    print(f"FP32 16x16x4 matrix-core throughput {t:.1f} TFLOP/s")
    assert 40.0 < t <= 157.3 * 1.02
