"""Edge cases of the pathwise adjoint (lll_plan_greeks / lll_plan_greeks_vjp).

* Zero volatility: every path keeps X = 0, so each price is a deterministic
  function of the initial forwards, P_i = s_i B(0,T_*) f_i(L(0,.)) with
  B(0,T_*) = B(0,T_1) / prod_l (1 + delta_l L(0,T_l)) (paper Section 3.3,
  eq. (caplet); the swaption payoff of the co-terminal swaps).  The deltas
  are then the derivatives of that closed form, taken here by FP64 central
  differences of the closed form itself (no derivation shared with the
  kernel).  Bar: 1e-5 relative to the row's largest entry (FP32 adjoint).
* Ragged path counts (1, 65 paths) against the oracle's common-random-number
  central differences, as in the full-structure tests (smaller bump).
"""
import numpy as np
import pytest

import workloads

from test_gpu_parity import _greeks_structure, _oracle_fd, _swaption_greeks_structure

pytestmark = pytest.mark.gpu


def _closed_form_prices(ts, L0):
    """FP64 prices (strike 0) at zero volatility for forwards L0."""
    d = ts.delta
    b = 1.0 + d * L0
    B0T = ts.B0_T1 / np.prod(b)
    K = ts.strikes[:, 0]
    N = len(L0)
    P = np.empty(N)
    for i in range(N):
        if ts.product == 0:
            D = np.prod(b[i + 1:])
            P[i] = d[i] * B0T * D * max(L0[i] - K[i], 0.0)
        else:
            Q = np.prod(b[i:])
            A = sum(d[l] * np.prod(b[l + 1:]) for l in range(i, N))
            P[i] = B0T * max(Q - 1.0 - K[i] * A, 0.0)
    return P


def _zero_vol_structure(N, product):
    L0 = 0.03 + 0.001 * np.arange(N)
    ts = workloads.make_structure(N, 0.25, L0, 3, lambda t, T, r: 0.0, [1.0],
                                  B0_T1=1.0 / (1.0 + 0.25 * 0.029))
    if product:
        ts = workloads.coterminal_swaptions(ts, [1.0])
    # alternate in and out of the money, 5% from the forward (swap) rate
    mult = 1.0 + 0.05 * np.where(np.arange(N) % 2 == 0, -1.0, 1.0)
    return ts.copy(strikes=ts.strikes * mult[:, None])


@pytest.mark.parametrize("product", [0, 1])
@pytest.mark.parametrize("N", [1, 9, 33])
def test_zero_vol_deltas_are_the_closed_form_derivatives(gpu_lib, product, N):
    ts = _zero_vol_structure(N, product)
    n = 1000
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
        plan.greeks(n, seed=1)
        g = plan.greeks_results()
        w = np.linspace(0.5, 1.5, N)
        plan.greeks_vjp(n, w, seed=1)
        r = plan.greeks_vjp_results()
    P = _closed_form_prices(ts, ts.L0)
    assert np.allclose(g["price"], P, rtol=1e-12, atol=1e-18)
    h = 1e-7
    J = np.empty((N, N))
    for l in range(N):
        up, dn = ts.L0.copy(), ts.L0.copy()
        up[l] += h
        dn[l] -= h
        J[:, l] = (_closed_form_prices(ts, up) - _closed_form_prices(ts, dn)) / (2 * h)
    scale = np.max(np.abs(J), axis=1, keepdims=True)
    assert np.all(np.abs(g["dP_dL0"] - J) <= 1e-5 * scale), (g["dP_dL0"], J)
    assert np.all(np.isfinite(g["dP_dvol"]))
    ref = w @ g["dP_dL0"]
    assert np.all(np.abs(r["vjp_L0"] - ref) <= 1e-5 * np.max(np.abs(ref)))


@pytest.mark.parametrize("product", [0, 1])
@pytest.mark.parametrize("n", [1, 65])
def test_greeks_ragged_path_counts(gpu_lib, oracle_mod, product, n):
    N, rtol = 4, 2e-3
    ts = _swaption_greeks_structure(N) if product else _greeks_structure(N)
    with gpu_lib.Plan(ts, precision=0, max_paths=256) as plan:
        plan.greeks(n, seed=1)
        g = plan.greeks_results()
    # h = 1e-9: with few paths a bump of 1e-6 can carry one path's payoff
    # across its strike, which moves the difference quotient by a sizeable
    # fraction of 1/n; FP64 paths resolve a 1e-9 bump to ~1e-7 relative
    JL, JV = _oracle_fd(oracle_mod, N, n, 1e-9, product=product)
    for got, ref in ((g["dP_dL0"], JL), (g["dP_dvol"], JV)):
        scale = np.max(np.abs(ref), axis=1, keepdims=True)
        assert np.all(np.abs(got - ref) <= rtol * np.abs(ref) + rtol * 1e-2 * scale + 1e-12), \
            (got, ref)
