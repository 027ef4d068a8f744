"""Black caplet quotes: the price formula against its textbook limits and
symmetries, and the implied volatility as its inverse."""
import math

import numpy as np

from paper_1006_3340_amd import quotes


def test_black_limits_and_parity():
    F, K, t, A = 0.04, 0.035, 2.5, 0.48
    # zero volatility: discounted intrinsic value; huge volatility: the forward
    assert quotes.black_caplet(F, K, 0.0, t, A) == A * (F - K)
    assert abs(quotes.black_caplet(F, K, 50.0, t, A) - A * F) < 1e-9
    # caplet - floorlet = A (F - K): the floorlet by the put form of Black's formula
    s = 0.3
    sq = s * math.sqrt(t)
    d1 = (math.log(F / K) + 0.5 * sq * sq) / sq
    N = lambda x: 0.5 * math.erfc(-x / math.sqrt(2))
    floor = A * (K * N(-(d1 - sq)) - F * N(-d1))
    assert abs(quotes.black_caplet(F, K, s, t, A) - floor - A * (F - K)) < 1e-15
    # at the money, small vol: price ~ A F sigma sqrt(t / 2 pi)
    p = quotes.black_caplet(F, F, 0.01, t, A)
    assert abs(p / (A * F * 0.01 * math.sqrt(t / (2 * math.pi))) - 1) < 1e-4


def test_implied_vol_inverts_black():
    rng = np.random.default_rng(3)
    for _ in range(200):
        F = rng.uniform(0.01, 0.08)
        K = F * rng.uniform(0.5, 1.6)
        t = rng.uniform(0.25, 10)
        s = rng.uniform(0.02, 1.0)
        p = quotes.black_caplet(F, K, s, t, 0.5)
        if p < 1e-14:
            continue
        assert abs(quotes.implied_vol(p, F, K, t, 0.5) - s) < 1e-9 * max(1.0, 1e-10 / p)
    # below intrinsic value: no volatility
    assert math.isnan(quotes.implied_vol(0.5 * 0.009, 0.04, 0.03, 1.0, 0.5))
