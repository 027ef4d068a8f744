"""LLL_EXACT: the FULL estimator with the drift of the exact subset expansion.

The expansion (paper Section 3.2, eq. (product)) and the oracle's quadrature
drift are the same drift: the oracle's is pinned to the subset sum to 1e-11
relative (test_oracle_drift.py::test_drift_vs_exact_subset_expansion).  So
the GPU's EXACT prices are compared with the oracle's FULL prices on the same
random numbers: FP64 plans to 1e-9 relative (the two drifts differ by the
rule's ~1e-11, FP64 arithmetic otherwise), FP32 plans at the FP32 bar of the
other schemes (1e-4, deep out-of-the-money floor as in _check_prices); per
path the FP64 EXACT fixings equal the FP64 FULL kernel's to 1e-10.
"""
import numpy as np
import pytest

import workloads

from test_gpu_parity import _check_prices

pytestmark = pytest.mark.gpu

FULL, EXACT = 0, 6
EINVAL, EUNSUPPORTED = -1, -5


@pytest.mark.parametrize("wl,n_paths", [("plain_n10", 5000), ("kluge_n9", 3001), ("gpu_n20", 300)])
def test_exact_fp64_matches_oracle_full(gpu_lib, oracle_mod, wl, n_paths):
    ts = workloads.WORKLOADS[wl]()
    ref = oracle_mod.Oracle(ts, seed=1).price(FULL, n_paths)
    with gpu_lib.Plan(ts, precision=1, max_paths=n_paths) as plan:
        plan.execute(EXACT, n_paths, seed=1)
        got = plan.results()
    assert np.all(np.abs(got["n_itm"] - ref["n_itm"]) <= 1)
    assert np.allclose(got["price"], ref["price"], rtol=1e-9, atol=1e-300)
    assert np.allclose(got["mart_resid"], ref["mart_resid"], rtol=0, atol=1e-11)


@pytest.mark.parametrize("wl,n_paths", [("plain_n10", 10000), ("gpu_n20", 2000), ("kluge_n9", 3001)])
def test_exact_fp32_matches_oracle_full(gpu_lib, oracle_mod, wl, n_paths):
    ts = workloads.WORKLOADS[wl]()
    ref = oracle_mod.Oracle(ts, seed=1).price(FULL, n_paths)
    with gpu_lib.Plan(ts, precision=0, max_paths=n_paths) as plan:
        plan.execute(EXACT, n_paths, seed=1)
        got = plan.results()
    _check_prices(got, ref, ts, 1e-4)


def test_exact_paths_equal_full_paths_fp64(gpu_lib):
    import torch
    ts = workloads.plain_fp64()
    n = 1000 + 13
    N = ts.n_rates
    fa = torch.empty((n, 2 * N), dtype=torch.float64, device="cuda")
    fb = torch.empty((n, 2 * N), dtype=torch.float64, device="cuda")
    with gpu_lib.Plan(ts, precision=1, max_paths=n) as plan:
        plan.execute(FULL, n, seed=4, path_fix=fa)
        plan.execute(EXACT, n, seed=4, path_fix=fb)
    torch.cuda.synchronize()
    fa, fb = fa.cpu().numpy(), fb.cpu().numpy()
    assert np.all(np.abs(fb / fa - 1.0) < 1e-10)


# The first rate's later rates as the kernel splits them: N = 1 (no coupling);
# low group only (N <= 6: 2, 5, 6); one padded column chunk (N = 9); 2, 4 and
# 8 chunks unrolled (N = 10, 11, 12: the table ring shorter than, equal to and
# inside one unrolled group); the prefix-product stack over 1 and 5 chunk bits
# (N = 13, 17); N = 20 itself.  FP64 plans (one 16-path tile per wavefront)
# and FP32 plans (two tiles), 517 paths (a ragged last wavefront).
@pytest.mark.parametrize("N,s", [(1, 3), (2, 2), (5, 2), (6, 2), (9, 1), (10, 1), (11, 1),
                                 (12, 1), (13, 1), (17, 1), (20, 1)])
@pytest.mark.parametrize("prec", [1, 0])
def test_exact_shapes(gpu_lib, oracle_mod, N, s, prec):
    ts = workloads.make_structure(N, 0.5, 0.02 + 0.002 * np.arange(N), s,
                                  workloads.exp_decay_vol(), [0.9, 1.0, 1.1])
    n = 517
    ref = oracle_mod.Oracle(ts, seed=2).price(FULL, n)
    with gpu_lib.Plan(ts, precision=prec, max_paths=n) as plan:
        plan.execute(EXACT, n, seed=2)
        got = plan.results()
    if prec == 1:
        assert np.allclose(got["price"], ref["price"], rtol=1e-9, atol=1e-300)
    else:
        _check_prices(got, ref, ts, 1e-4)


def test_exact_brownian_and_zero_vol(gpu_lib, oracle_mod):
    tb = workloads.brownian(N=6)
    ref = oracle_mod.Oracle(tb, seed=1).price(FULL, 3000)
    with gpu_lib.Plan(tb, precision=1, max_paths=3000) as plan:
        plan.execute(EXACT, 3000)
        assert np.allclose(plan.results()["price"], ref["price"], rtol=1e-10, atol=1e-300)
    ts = workloads.make_structure(7, 0.5, 0.03 + 0.004 * np.arange(7), 4, lambda t, T, r: 0.0,
                                  [0.7, 1.0, 1.3])
    B = ts.B0_T1 / np.cumprod(1.0 + ts.delta * ts.L0)
    exact = ts.delta[:, None] * B[:, None] * np.maximum(ts.L0[:, None] - ts.strikes, 0.0)
    for prec in (0, 1):
        with gpu_lib.Plan(ts, precision=prec, max_paths=300) as plan:
            plan.execute(EXACT, 300)
            assert np.allclose(plan.results()["price"], exact, rtol=1e-12, atol=1e-18)


def test_exact_swaptions(gpu_lib, oracle_mod):
    ts = workloads.coterminal_swaptions(workloads.plain_fp64(), [0.8, 1.0, 1.2])
    ref = oracle_mod.Oracle(ts, seed=3).price(FULL, 4000)
    for prec, rtol in ((1, 1e-9), (0, 1e-4)):
        with gpu_lib.Plan(ts, precision=prec, max_paths=4000) as plan:
            plan.execute(EXACT, 4000, seed=3)
            got = plan.results()
        _check_prices(got, ref, ts, rtol)


def test_exact_errors(gpu_lib):
    ts = workloads.make_structure(21, 0.25, 0.03, 1, workloads.exp_decay_vol(), [1.0])
    with gpu_lib.Plan(ts, precision=0, max_paths=64) as plan:
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.execute(EXACT, 64)
        assert ei.value.code == EUNSUPPORTED
        plan.execute(FULL, 64)                     # the plan is still usable
    with gpu_lib.Batch([workloads.plain_fp64()], max_paths_each=64) as bt:
        with pytest.raises(gpu_lib.LLLError) as ei:
            bt.execute(EXACT, 64)
        assert ei.value.code == EINVAL


def test_exact_bench_size_sampled_paths_and_reduction(gpu_lib, oracle_mod):
    """The launch the bench times (N = 20, 2^16 paths, FP32, one period launch
    per fixing on the matrix cores): sampled per-path fixings against the
    oracle's FULL paths (whose drift equals the subset expansion to 1e-11) at
    the FP32 path tolerance, the first and last path included, and the
    reduction against the mean of the per-path payoffs recomputed on the host."""
    import torch
    ts = workloads.gpu_scale()
    n = 1 << 16
    o = oracle_mod.Oracle(ts, seed=1)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(n, size=12, replace=False))
    sample[0], sample[-1] = 0, n - 1
    fix = torch.empty((n, 2 * ts.n_rates), dtype=torch.float64, device="cuda")
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
        plan.execute(EXACT, n, seed=1, path_fix=fix)
        got = plan.results()
    torch.cuda.synchronize()
    f = fix.cpu().numpy()
    Lg, Dg = f[:, 0::2], f[:, 1::2]
    Lo, Do = o.paths(FULL, sample)
    assert np.all(np.abs(Lg[sample] / Lo - 1.0) < 2e-5)
    assert np.all(np.abs(Dg[sample] / Do - 1.0) < 2e-5)
    pay = Dg[:, :, None] * np.maximum(Lg[:, :, None] - ts.strikes[None], 0.0)
    B0T = ts.B0_T1 / np.prod(1.0 + ts.delta * ts.L0)
    host_price = ts.delta[:, None] * B0T * pay.mean(axis=0)
    assert np.allclose(got["price"], host_price, rtol=1e-12, atol=0)


@pytest.mark.parametrize("wl,prec,n", [("gpu_n20", 0, 1 << 16), ("plain_n10", 1, 4096)])
def test_exact_deterministic_and_split_range(gpu_lib, wl, prec, n):
    """Repeat runs are bit-identical, and two half-range runs (path offsets 0
    and n/2, whole wavefronts) give the same per-wavefront partials as the
    whole run: a path's draws depend only on its global index, its state on
    nothing shared with other paths."""
    ts = workloads.WORKLOADS[wl]()
    with gpu_lib.Plan(ts, precision=prec, max_paths=n) as plan:
        plan.execute(EXACT, n, seed=7)
        a, pa = plan.sums(), plan.partials()
        plan.execute(EXACT, n, seed=7)
        b, pb = plan.sums(), plan.partials()
        assert np.array_equal(a, b) and np.array_equal(pa, pb)
        half = n // 2
        plan.execute(EXACT, half, seed=7, path_offset=0)
        p1 = plan.partials()
        plan.execute(EXACT, half, seed=7, path_offset=half)
        p2 = plan.partials()
        assert np.array_equal(np.concatenate([p1, p2]), pa)
        plan.execute(EXACT, n, seed=8)
        assert not np.array_equal(plan.sums(), a)
