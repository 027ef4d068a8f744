"""Black (1976) quotes of caplet prices: implied volatilities (host side).

Markets quote caplets by the volatility that Black's formula needs to
reproduce their price; the paper compares its schemes by the difference of
these implied volatilities in basis points (Section 4).  Caplet r (0-based)
pays delta_r (L(T, T) - K)^+ at the end of its accrual period, fixes at
tenor[r], and its forward is L(0, T) = L0[r]; its discounted Black price is
    delta_r B(0, T_pay) [F N(d1) - K N(d2)],  d1,2 = (ln(F/K) +- sigma^2 t / 2) / (sigma sqrt t),
with B(0, T_pay) = B(0, T_1) / prod_{l <= r} (1 + delta_l L0_l).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["black_caplet", "implied_vol", "caplet_implied_vols"]


def _ncdf(x: float) -> float:
    return 0.5 * math.erfc(-x / math.sqrt(2.0))


def black_caplet(F: float, K: float, sigma: float, t: float, annuity: float) -> float:
    """annuity x Black(F, K, sigma, t); annuity = delta B(0, T_pay)."""
    if sigma <= 0.0 or t <= 0.0:
        return annuity * max(F - K, 0.0)
    s = sigma * math.sqrt(t)
    d1 = (math.log(F / K) + 0.5 * s * s) / s
    return annuity * (F * _ncdf(d1) - K * _ncdf(d1 - s))


def implied_vol(price: float, F: float, K: float, t: float, annuity: float,
                lo: float = 1e-6, hi: float = 5.0, tol: float = 1e-13) -> float:
    """Volatility with black_caplet(...) = price by bisection on [lo, hi] (the
    price is increasing in sigma); NaN if the price is outside the prices of
    [lo, hi] (e.g. below intrinsic value)."""
    p_lo = black_caplet(F, K, lo, t, annuity)
    p_hi = black_caplet(F, K, hi, t, annuity)
    if not (p_lo <= price <= p_hi):
        return float("nan")
    a, b = lo, hi
    for _ in range(200):
        m = 0.5 * (a + b)
        if black_caplet(F, K, m, t, annuity) < price:
            a = m
        else:
            b = m
        if b - a < tol:
            break
    return 0.5 * (a + b)


def caplet_implied_vols(ts, price: np.ndarray) -> np.ndarray:
    """Implied volatilities [N][S] of caplet prices [N][S] of term structure ts
    (NaN where a price has no Black volatility)."""
    L0 = np.asarray(ts.L0, dtype=np.float64)
    delta = np.asarray(ts.delta, dtype=np.float64)
    B_pay = ts.B0_T1 / np.cumprod(1.0 + delta * L0)
    out = np.full(np.shape(price), np.nan)
    for r in range(len(L0)):
        for j in range(price.shape[1]):
            out[r, j] = implied_vol(float(price[r, j]), float(L0[r]), float(ts.strikes[r, j]),
                                    float(ts.tenor[r]), float(delta[r] * B_pay[r]))
    return out
