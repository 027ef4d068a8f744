"""The allocation-free entry point lll_price_caplets_static against
lll_price_caplets: the same kernels on buffers carved from the library's
static device workspace, so the prices must be the same numbers bit for bit.
Two calls in a row share the workspace; the second is smaller (fewer rates,
steps, strikes and paths), so stale contents of the first would show."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _same(lll, ts, n, scheme, precision):
    print(f"static workspace: {ts.name} N={ts.n_rates} paths={n} scheme={scheme} "
          f"precision={precision}", flush=True)
    a = lll.price_caplets_static(ts, n, scheme, seed=1, precision=precision)
    b = lll.price_caplets(ts, n, scheme, seed=1, precision=precision)
    for key in ("price", "stderr", "mart_resid"):
        assert np.array_equal(a[key], b[key]), (key, np.max(np.abs(a[key] - b[key])))
    assert np.all(np.isfinite(a["price"])) and np.any(a["price"] > 0)


def test_static_workspace_matches_plan_path_two_calls(gpu_lib):
    lll = gpu_lib
    # the benchmark workload at full size (N = 20, 400 steps, 2^20 paths), then
    # a smaller one (N = 10, 100 steps, one strike, a ragged path count)
    _same(lll, workloads.gpu_scale(), 1 << 20, lll.FULL, lll.FP32)
    _same(lll, workloads.plain_fp64(), 10000 - 37, lll.PICARD, lll.FP32)


def test_static_workspace_schemes_and_precisions(gpu_lib):
    lll = gpu_lib
    ts = workloads.plain_fp64()
    for scheme in (lll.FULL, lll.PICARD, lll.FROZEN, lll.FIRST_ORDER, lll.SECOND_ORDER):
        _same(lll, ts, 4097, scheme, lll.FP64)
    sw = workloads.coterminal_swaptions(workloads.gpu_scale(), [0.8, 1.0, 1.2])
    _same(lll, sw, 3000, lll.FULL, lll.FP32)
    _same(lll, workloads.learned_drift(), 1 << 16, lll.PICARD, lll.FP32)


def test_static_workspace_rejects_oversize_and_other_schemes(gpu_lib):
    lll = gpu_lib
    with pytest.raises(lll.LLLError) as ei:
        lll.price_caplets_static(workloads.learned_drift(), 1 << 20, lll.FULL)
    assert ei.value.code == -1 and "static workspace holds" in str(ei.value)
    with pytest.raises(lll.LLLError) as ei:
        lll.price_caplets_static(workloads.plain_fp64(), 64, lll.EXACT)
    assert ei.value.code == -5
    # a rejected call leaves the workspace usable
    _same(lll, workloads.plain_fp64(), 640, lll.FULL, lll.FP32)
