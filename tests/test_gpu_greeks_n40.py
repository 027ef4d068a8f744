"""Pathwise Greeks of the N = 40 quarterly workload (the 40-slot adjoint
kernels: forward pass with the state in LDS, per-caplet sweeps, per-period
vector-Jacobian product) against central finite differences of the FP64
oracle's FULL prices under common random numbers (same Philox streams, same
paths), for the input columns l = 0, 20, 39 (L(0, T_l) and the vol level
v_l), with B(0, T_1) and the absolute strikes held.

Bars: with h = 1e-6 the central difference of the FP64 oracle is the
pathwise derivative up to O(h^2) and to the paths whose payoff kink lies
within the bump (none expected at 2000 paths), so the FP32 adjoint must match
to 2e-3 relative (plus 2e-5 of the row's largest entry for entries that
vanish); with h = 1e-4 a few paths cross the strike inside the bump: 3e-2.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

FULL = 0
COLUMNS = (0, 20, 39)


def _bumped(base, l, kind, h):
    levels = np.full(base.n_rates, 0.12)
    L0 = base.L0.copy()
    (L0 if kind == "L" else levels)[l] += h
    return workloads.adjoint_greeks(levels=levels, L0=L0).copy(B0_T1=base.B0_T1,
                                                               strikes=base.strikes.copy())


def _oracle_fd(oracle_mod, base, n, h):
    fd = {}
    for l in COLUMNS:
        for kind in ("L", "v"):
            up = oracle_mod.Oracle(_bumped(base, l, kind, +h), seed=1).price(FULL, n)["price"][:, 0]
            dn = oracle_mod.Oracle(_bumped(base, l, kind, -h), seed=1).price(FULL, n)["price"][:, 0]
            fd[(kind, l)] = (up - dn) / (2 * h)
    return fd


@pytest.fixture(scope="module")
def gpu_greeks(gpu_lib):
    base = workloads.adjoint_greeks()
    n = 2000
    rng = np.random.default_rng(8)
    w = rng.normal(0.0, 1.0, base.n_rates)
    with gpu_lib.Plan(base, precision=0, max_paths=n) as plan:
        plan.greeks(n, seed=1)
        g = plan.greeks_results()
        plan.greeks_vjp(n, w, seed=1)
        v = plan.greeks_vjp_results()
    return base, n, g, w, v


@pytest.mark.parametrize("h,rtol", [(1e-6, 2e-3), (1e-4, 3e-2)])
def test_n40_greeks_match_oracle_finite_differences(gpu_lib, oracle_mod, gpu_greeks, h, rtol):
    base, n, g, w, v = gpu_greeks
    print(f"N=40 Greeks vs FP64 oracle central differences h={h} paths={n}", flush=True)
    fd = _oracle_fd(oracle_mod, base, n, h)
    worst = 0.0
    for (kind, l), ref in fd.items():
        got = (g["dP_dL0"] if kind == "L" else g["dP_dvol"])[:, l]
        scale = np.max(np.abs(ref))
        err = np.abs(got - ref)
        assert np.all(err <= rtol * np.abs(ref) + rtol * 1e-2 * scale), (kind, l, got, ref)
        big = np.abs(ref) > 1e-2 * scale
        worst = max(worst, float(np.max(err[big] / np.abs(ref[big]))))
        # the single reverse sweep seeded with w gives w^T J on the same paths
        vj = v["vjp_L0"] if kind == "L" else v["vjp_vol"]
        bound = rtol * (np.abs(w) @ np.abs(ref) + 1e-2 * scale * np.abs(w).sum())
        assert abs(vj[l] - w @ ref) <= bound, (kind, l, vj[l], w @ ref)
    print(f"max relative error (entries above 1% of their column): {worst:.2e}")
    ref_price = oracle_mod.Oracle(base, seed=1).price(FULL, n)["price"][:, 0]
    assert np.allclose(g["price"], ref_price, rtol=1e-4)
    assert np.allclose(v["price"], ref_price, rtol=1e-4)
