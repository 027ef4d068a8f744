"""Single-sweep vector-Jacobian product of the caplet and swaption prices (lll_plan_greeks_vjp).

It seeds one reverse sweep with the weights g_i at every fixing date, so it
must equal g^T J of the per-caplet sweeps (lll_plan_greeks, pinned against the
oracle's finite differences and the Fourier price in test_gpu_parity.py) up to
FP32 summation order: the state adjoints of all caplets are summed in FP32
during the sweep instead of per caplet.  Tolerance 1e-5 of the largest entry
of g^T J (FP32 accumulation over K = N s steps of terms of one sign).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _check(got, ref, tol=1e-5):
    scale = np.max(np.abs(ref))
    assert np.all(np.abs(got - ref) <= tol * scale), (np.max(np.abs(got - ref)) / scale, got, ref)


@pytest.mark.parametrize("wl,n,product", [("adjoint_n40", 1 << 16, 0), ("plain_n10", 4096, 0),
                                          ("gpu_n20", 4096, 0), ("adjoint_n40", 1 << 16, 1),
                                          ("gpu_n20", 4096, 1)])
def test_vjp_equals_weighted_jacobian(gpu_lib, wl, n, product):
    ts = workloads.WORKLOADS[wl]()
    N = ts.n_rates
    if product == 1:
        ts = workloads.coterminal_swaptions(ts, [1.0])
    if ts.n_strikes > 1:
        ts = ts.copy(strikes=ts.strikes[:, 1:2].copy())   # ATM as strike 0
    rng = np.random.default_rng(7)
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
        plan.greeks(n, seed=3)
        g = plan.greeks_results()
        for w in (rng.normal(size=N), np.eye(N)[N // 2], np.eye(N)[N - 1], np.ones(N)):
            plan.greeks_vjp(n, w, seed=3)
            r = plan.greeks_vjp_results()
            assert np.allclose(r["price"], g["price"], rtol=1e-12, atol=0)
            _check(r["vjp_L0"], w @ g["dP_dL0"])
            _check(r["vjp_vol"], w @ g["dP_dvol"])


@pytest.mark.parametrize("N,s", [(1, 3), (2, 1), (9, 2), (17, 1)])
def test_vjp_shapes(gpu_lib, N, s):
    ts = workloads.make_structure(N, 0.25, 0.02 + 0.001 * np.arange(N), s,
                                  workloads.exp_decay_vol(), [1.0])
    n = 2048 + 17
    w = np.linspace(-1.0, 2.0, N)
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
        plan.greeks(n, seed=2)
        g = plan.greeks_results()
        plan.greeks_vjp(n, w, seed=2)
        r = plan.greeks_vjp_results()
    _check(r["vjp_L0"], w @ g["dP_dL0"])
    _check(r["vjp_vol"], w @ g["dP_dvol"])


def test_vjp_full_size_and_timing(gpu_lib):
    """N = 40, 2^20 paths: the vector-Jacobian product against g^T J, and its
    cost against the full Jacobian's (one sweep instead of N)."""
    ts = workloads.adjoint_greeks()
    N, n = ts.n_rates, 1 << 20
    w = np.linspace(1.0, 2.0, N)
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
        plan.set_timing(True)
        plan.greeks(n, seed=1)
        g = plan.greeks_results()
        t_jac = plan.timing()["paths"]
        plan.greeks_vjp(n, w, seed=1)
        r = plan.greeks_vjp_results()
        t_vjp = plan.timing()["paths"]
    _check(r["vjp_L0"], w @ g["dP_dL0"])
    _check(r["vjp_vol"], w @ g["dP_dvol"])
    print(f"full Jacobian {t_jac:.1f} ms, vector-Jacobian product {t_vjp:.1f} ms")
    assert t_vjp < t_jac / 4


def test_vjp_errors(gpu_lib):
    ts = workloads.plain_fp64()
    with gpu_lib.Plan(ts, precision=0, max_paths=64) as plan:
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.greeks_vjp(64, np.full(ts.n_rates, np.nan))
        assert ei.value.code == -1
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.greeks_vjp_results()                 # nothing run yet
        assert ei.value.code == -1
    with gpu_lib.Plan(ts, precision=1, max_paths=64) as plan:   # FP64 plan
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.greeks_vjp(64, np.ones(ts.n_rates))
        assert ei.value.code == -5
