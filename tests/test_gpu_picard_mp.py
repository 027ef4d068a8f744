"""PICARD in the maturity-parallel layout (LLL_PICARD_MP) through the C ABI.

It is the PICARD estimator (paper Section 3, eqs. (Picard-2), (bdrift)) with
the drift integrals of all accrual periods computed at once, so its parity
bar is the FP32 PICARD bar against the oracle's PICARD: 1e-4 relative per
caplet where the oracle has at least 100 in-the-money paths, else 1e-4 of the
at-the-money price of that caplet.  Against the FP32 path kernel's PICARD the
predictor is bitwise the same (same FP32 updates); the main state is the same
sum in another order (per period, the nodes summed in a tree), so the
per-path fixings agree to FP32 accumulation error over the K steps: 2e-5
relative, as for the FP32 kernels against the FP64 oracle.
"""
import numpy as np
import pytest

import workloads

from test_gpu_parity import _check_prices

pytestmark = pytest.mark.gpu

PICARD, PICARD_MP = 1, 5
EUNSUPPORTED = -5


@pytest.mark.parametrize("wl,n_paths", [("plain_n10", 10000), ("gpu_n20", 4173),
                                        ("kluge_n9", 3001), ("mlp_n40", 700),
                                        ("mp_n60", 517)])
def test_mp_matches_oracle_picard(gpu_lib, oracle_mod, wl, n_paths):
    ts = workloads.WORKLOADS[wl]()
    ref = oracle_mod.Oracle(ts, seed=1).price(PICARD, n_paths)
    with gpu_lib.Plan(ts, precision=0, max_paths=n_paths) as plan:
        plan.execute(PICARD_MP, n_paths, seed=1)
        got = plan.results()
    _check_prices(got, ref, ts, 1e-4)
    assert np.all(np.abs(got["n_itm"] - ref["n_itm"]) <= 3 + 1e-4 * n_paths)
    fwd = np.cumprod((1.0 + ts.delta * ts.L0)[::-1])[::-1]   # prod_{l>=r}(1 + delta L0)
    assert np.all(np.abs(got["mart_resid"] - ref["mart_resid"]) <= 1e-4 * fwd)


@pytest.mark.parametrize("wl", ["plain_n10", "gpu_n20", "kluge_n9", "mlp_n40"])
def test_mp_matches_path_kernel_picard(gpu_lib, wl):
    import torch
    ts = workloads.WORKLOADS[wl]()
    n = 4096 + 37
    N = ts.n_rates
    fa = torch.empty((n, 2 * N), dtype=torch.float64, device="cuda")
    fb = torch.empty((n, 2 * N), dtype=torch.float64, device="cuda")
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
        plan.execute(PICARD, n, seed=5, path_fix=fa)
        a = plan.results()
        plan.execute(PICARD_MP, n, seed=5, path_fix=fb)
        b = plan.results()
    torch.cuda.synchronize()
    fa, fb = fa.cpu().numpy(), fb.cpu().numpy()
    assert np.all(np.abs(fb / fa - 1.0) < 2e-5)
    _check_prices(b, a, ts, 2e-5)


def test_mp_full_size(gpu_lib, oracle_mod):
    """The few-paths / many-rates configuration itself (N = 60, 10^4 paths):
    every caplet against the oracle's PICARD on the same 10^4 paths, sampled
    per-path fixings, and the reduction against the host mean of the per-path
    payoffs."""
    import torch
    ts = workloads.maturity_parallel()
    n = 10000
    o = oracle_mod.Oracle(ts, seed=1)
    fix = torch.empty((n, 2 * ts.n_rates), dtype=torch.float64, device="cuda")
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
        plan.execute(PICARD_MP, n, seed=1, path_fix=fix)
        got = plan.results()
    torch.cuda.synchronize()
    f = fix.cpu().numpy()
    Lg, Dg = f[:, 0::2], f[:, 1::2]
    rng = np.random.default_rng(4)
    sample = np.sort(rng.choice(n, size=24, replace=False))
    sample[0], sample[-1] = 0, n - 1
    Lo, Do = o.paths(PICARD, sample)
    assert np.all(np.abs(Lg[sample] / Lo - 1.0) < 2e-5)
    assert np.all(np.abs(Dg[sample] / Do - 1.0) < 2e-5)
    pay = Dg[:, :, None] * np.maximum(Lg[:, :, None] - ts.strikes[None], 0.0)
    B0T = ts.B0_T1 / np.prod(1.0 + ts.delta * ts.L0)
    assert np.allclose(got["price"], ts.delta[:, None] * B0T * pay.mean(axis=0), rtol=1e-12, atol=0)
    _check_prices(got, o.price(PICARD, n), ts, 1e-4)


def test_mp_chunks_deterministic_and_split_range(gpu_lib):
    """2^15 paths at N = 60 run in two chunks of the 2 GiB buffers: the wave
    partials are bitwise those of two half-range calls and of a repeat."""
    ts = workloads.maturity_parallel()
    n = 1 << 15
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
        plan.execute(PICARD_MP, n, seed=3)
        a, pa = plan.sums(), plan.partials()
        plan.execute(PICARD_MP, n, seed=3)
        assert np.array_equal(plan.partials(), pa) and np.array_equal(plan.sums(), a)
        half = n // 2
        plan.execute(PICARD_MP, half, seed=3, path_offset=0)
        p1 = plan.partials()
        plan.execute(PICARD_MP, half, seed=3, path_offset=half)
        p2 = plan.partials()
        assert np.array_equal(np.concatenate([p1, p2]), pa)


# s > 16 splits a period into equal step chunks (17 -> 9 + 8 with one padded
# step, 33 -> 3 x 11, 35 -> 12 + 12 + 11)
@pytest.mark.parametrize("N,s", [(1, 1), (1, 7), (2, 1), (9, 3), (17, 2), (41, 2), (64, 1),
                                 (5, 17), (3, 33), (4, 35)])
def test_mp_shapes(gpu_lib, oracle_mod, N, s):
    ts = workloads.make_structure(N, 0.25, 0.02 + 0.001 * np.arange(N), s,
                                  workloads.exp_decay_vol(), [0.9, 1.0, 1.1])
    ref = oracle_mod.Oracle(ts, seed=1).price(PICARD, 999)
    with gpu_lib.Plan(ts, precision=0, max_paths=999) as plan:
        plan.execute(PICARD_MP, 999, seed=1)
        got = plan.results()
    _check_prices(got, ref, ts, 1e-4)


@pytest.mark.parametrize("n_paths", [1, 63, 65, 257])
def test_mp_ragged_path_counts(gpu_lib, oracle_mod, n_paths):
    ts = workloads.plain_fp64()
    ref = oracle_mod.Oracle(ts, seed=1).price(PICARD, n_paths)
    with gpu_lib.Plan(ts, precision=0, max_paths=1024) as plan:
        plan.execute(PICARD_MP, n_paths, seed=1)
        got = plan.results()
    _check_prices(got, ref, ts, 1e-4)
    assert np.all(np.abs(got["n_itm"] - ref["n_itm"]) <= 1)


def test_mp_zero_vol_is_exact(gpu_lib):
    ts = workloads.make_structure(47, 0.25, 0.03 + 0.0004 * np.arange(47), 3,
                                  lambda t, T, r: 0.0, [0.7, 1.0, 1.3])
    B = ts.B0_T1 / np.cumprod(1.0 + ts.delta * ts.L0)
    exact = ts.delta[:, None] * B[:, None] * np.maximum(ts.L0[:, None] - ts.strikes, 0.0)
    with gpu_lib.Plan(ts, precision=0, max_paths=300) as plan:
        plan.execute(PICARD_MP, 300)
        assert np.allclose(plan.results()["price"], exact, rtol=1e-12, atol=1e-18)


def test_mp_swaptions(gpu_lib, oracle_mod):
    ts = workloads.coterminal_swaptions(workloads.maturity_parallel())
    n = 2000
    ref = oracle_mod.Oracle(ts, seed=2).price(PICARD, n)
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
        plan.execute(PICARD_MP, n, seed=2)
        got = plan.results()
    _check_prices(got, ref, ts, 1e-4)


def test_mp_errors(gpu_lib):
    big = workloads.maturity_parallel()
    with gpu_lib.Plan(big, precision=0, max_paths=64) as plan:
        for scheme in (0, 1, 2, 3, 4):        # the path-per-lane kernels stop at 40 rates
            with pytest.raises(gpu_lib.LLLError) as ei:
                plan.execute(scheme, 64)
            assert ei.value.code == EUNSUPPORTED
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.greeks(64)
        assert ei.value.code == EUNSUPPORTED
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.drift(0, big.L0)
        assert ei.value.code == EUNSUPPORTED
        plan.execute(PICARD_MP, 64)
        assert np.all(np.isfinite(plan.results()["price"]))
    with gpu_lib.Plan(workloads.plain_fp64(), precision=1, max_paths=64) as plan:
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.execute(PICARD_MP, 64)
        assert ei.value.code == EUNSUPPORTED
    with gpu_lib.Plan(workloads.brownian(N=6), precision=0, max_paths=64) as plan:
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.execute(PICARD_MP, 64)
        assert ei.value.code == EUNSUPPORTED
