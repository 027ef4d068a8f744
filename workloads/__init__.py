"""Seeded synthetic workloads for the Lévy LIBOR Monte Carlo path.

This module only *constructs inputs*: tenor grids, initial forward rates,
volatility tables, driver parameters and strike grids.  It holds none of the
method's arithmetic (no drift, no sampling, no pricing), so that both the
FP64 CPU oracle and the HIP path can be fed from it without sharing code.

Conventions (paper Section 2, tenor structure 0 = T_0 < T_1 < ... < T_N <
T_{N+1} = T_*):

* rates are 0-indexed in arrays: slot ``r`` holds the paper's rate
  ``i = r + 1`` with maturity ``T_i``; ``delta[r] = T_{i+1} - T_i``;
* the Euler grid has ``steps_per_period`` equal steps inside each accrual
  period [T_m, T_{m+1}], m = 0..N-1 (T_0 = 0), so that every T_i is hit;
* ``vol[k, r]`` is lambda(t_k, T_{r+1}) at the left point t_k of step k; the
  entries of rates already fixed (T_{r+1} <= t_k) are never read and are 0;
* ``strikes[r, j]`` is the j-th absolute strike of the caplet on rate r.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

DRIVER_NIG = 0
DRIVER_BROWNIAN = 1

SCHEME_FULL = 0
SCHEME_PICARD = 1
SCHEME_FROZEN = 2
SCHEME_MLP = 3

SCHEME_NAMES = {"full": SCHEME_FULL, "picard": SCHEME_PICARD,
                "frozen": SCHEME_FROZEN, "mlp": SCHEME_MLP}

N_MAX = 40       # path-per-lane kernels
N_MAX_MP = 64    # the maturity-parallel PICARD layout


@dataclasses.dataclass
class TermStructure:
    """One Lévy LIBOR term structure plus its caplet strikes."""

    tenor: np.ndarray          # T_1..T_N, shape [N]
    delta: np.ndarray          # delta_1..delta_N, shape [N]
    L0: np.ndarray             # L(0, T_i), shape [N]
    B0_T1: float               # B(0, T_1)
    steps_per_period: int      # s
    vol: np.ndarray            # lambda(t_k, T_i), shape [N*s, N]
    strikes: np.ndarray        # shape [N, S]
    driver: int = DRIVER_NIG
    alpha: float = 18.0
    beta: float = -4.0
    delta_nig: float = 1.0
    c: float = 0.0             # Brownian variance rate (driver == BROWNIAN)
    struct_id: int = 0         # fourth Philox counter word (low 24 bits)
    name: str = ""
    product: int = 0           # 0: caplets; 1: co-terminal payer swaptions

    @property
    def n_rates(self) -> int:
        return int(self.tenor.shape[0])

    @property
    def n_steps(self) -> int:
        return self.n_rates * self.steps_per_period

    @property
    def n_strikes(self) -> int:
        return int(self.strikes.shape[1])

    def validate_shapes(self) -> None:
        N, s = self.n_rates, self.steps_per_period
        assert self.delta.shape == (N,)
        assert self.L0.shape == (N,)
        assert self.vol.shape == (N * s, N)
        assert self.strikes.ndim == 2 and self.strikes.shape[0] == N

    def copy(self, **changes) -> "TermStructure":
        fields = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}
        for k, v in fields.items():
            if isinstance(v, np.ndarray):
                fields[k] = v.copy()
        fields.update(changes)
        return TermStructure(**fields)


def step_times(tenor: np.ndarray, steps_per_period: int) -> np.ndarray:
    """Left points t_k of the Euler grid (input construction only)."""
    T = np.concatenate([[0.0], np.asarray(tenor, dtype=np.float64)])
    s = steps_per_period
    t = np.empty(len(tenor) * s)
    for m in range(len(tenor)):
        for j in range(s):
            t[m * s + j] = T[m] + j * (T[m + 1] - T[m]) / s
    return t


def vol_table(tenor: np.ndarray, steps_per_period: int,
              fn: Callable[[float, float, int], float]) -> np.ndarray:
    """Tabulate lambda(t_k, T_i) = fn(t_k, T_i, r) on the grid; 0 for fixed rates."""
    N = len(tenor)
    t = step_times(tenor, steps_per_period)
    vol = np.zeros((N * steps_per_period, N))
    for k, tk in enumerate(t):
        for r in range(N):
            if tenor[r] > tk + 1e-12:
                vol[k, r] = fn(tk, tenor[r], r)
    return vol


def exp_decay_vol(level: float = 0.12, amp: float = 0.1, decay: float = 0.5,
                  levels: Optional[np.ndarray] = None):
    """lambda(t, T_i) = v_i + amp * exp(-decay (T_i - t)) with v_i = level (or levels[i])."""
    def fn(t, T, r):
        v = level if levels is None else float(levels[r])
        return v + amp * math.exp(-decay * (T - t))
    return fn


def flat_extension_B0(tenor: np.ndarray, L0: np.ndarray) -> float:
    """B(0, T_1) = 1 / (1 + T_1 L(0, T_1)) when only forwards are given."""
    return 1.0 / (1.0 + float(tenor[0]) * float(L0[0]))


def make_structure(N: int, delta: float, L0, steps_per_period: int, vol_fn,
                   strike_mult, alpha=18.0, beta=-4.0, delta_nig=1.0,
                   driver=DRIVER_NIG, c=0.0, struct_id=0, name="",
                   B0_T1: Optional[float] = None) -> TermStructure:
    tenor = delta * np.arange(1, N + 1, dtype=np.float64)
    dl = np.full(N, float(delta))
    L0 = np.broadcast_to(np.asarray(L0, dtype=np.float64), (N,)).copy()
    vol = vol_table(tenor, steps_per_period, vol_fn)
    mult = np.atleast_1d(np.asarray(strike_mult, dtype=np.float64))
    strikes = L0[:, None] * mult[None, :]
    if B0_T1 is None:
        B0_T1 = flat_extension_B0(tenor, L0)
    ts = TermStructure(tenor=tenor, delta=dl, L0=L0, B0_T1=float(B0_T1),
                       steps_per_period=int(steps_per_period), vol=vol,
                       strikes=strikes, driver=driver, alpha=float(alpha),
                       beta=float(beta), delta_nig=float(delta_nig), c=float(c),
                       struct_id=int(struct_id), name=name)
    ts.validate_shapes()
    return ts


# ---------------------------------------------------------------------------
# The five workloads of the build (plain method, GPU scale, batched, learned
# drift, adjoint) and the paper's own numerical example.
# ---------------------------------------------------------------------------

def plain_fp64() -> TermStructure:
    """N=10 semiannual rates (T_N = 5y), flat 4%, constant vol 0.15, NIG(18,-4,1),
    10 Euler steps per period, ATM caplets."""
    return make_structure(10, 0.5, 0.04, 10, lambda t, T, r: 0.15, [1.0],
                          name="plain_n10")


def gpu_scale() -> TermStructure:
    """N=20 semiannual (10y), L0_i = 0.03 + 0.002 i, lambda = 0.12 + 0.1 e^{-0.5(T_i - t)},
    NIG(18,-4,1), 20 steps per period, strikes {0.8, 1.0, 1.2} x forward."""
    L0 = 0.03 + 0.002 * np.arange(1, 21)
    return make_structure(20, 0.5, L0, 20, exp_decay_vol(), [0.8, 1.0, 1.2],
                          name="gpu_n20")


def learned_drift() -> TermStructure:
    """N=40 quarterly (10y), L0_i = 0.03 + 0.001 i, same vol formula, NIG(18,-4,1),
    10 steps per period (dt = 0.025), strikes {0.8, 1.0, 1.2} x forward."""
    L0 = 0.03 + 0.001 * np.arange(1, 41)
    return make_structure(40, 0.25, L0, 10, exp_decay_vol(), [0.8, 1.0, 1.2],
                          name="mlp_n40")


def maturity_parallel() -> TermStructure:
    """Few paths, many rates: N=60 quarterly (15y), L0_i = 0.03 + 0.0005 i, the
    exp-decay vol, NIG(18,-4,1), 10 steps per period, strikes {0.8, 1.0, 1.2} x
    forward; priced with 10^4 paths."""
    L0 = 0.03 + 0.0005 * np.arange(1, 61)
    return make_structure(60, 0.25, L0, 10, exp_decay_vol(), [0.8, 1.0, 1.2],
                          name="mp_n60")


def adjoint_greeks(levels: Optional[np.ndarray] = None,
                   L0: Optional[np.ndarray] = None) -> TermStructure:
    """N=40 quarterly, ATM caplets; vol lambda = v_i + 0.1 e^{-0.5(T_i - t)} with
    vol levels v_i (0.12 by default) as differentiable inputs."""
    if L0 is None:
        L0 = 0.03 + 0.001 * np.arange(1, 41)
    if levels is None:
        levels = np.full(40, 0.12)
    return make_structure(40, 0.25, L0, 10, exp_decay_vol(levels=levels), [1.0],
                          name="adjoint_n40")


def batched(n_structures: int = 64, seed: int = 1) -> List[TermStructure]:
    """64 independent term structures drawn with numpy PCG64(seed):
    N ~ U{8..40}, delta in {0.25, 0.5}, L0 ~ U[0.01, 0.06] per rate,
    alpha ~ U[12, 25], beta ~ U[-5, 0], delta_NIG ~ U[0.5, 1.5];
    vol by the exp-decay formula, dt = 0.025, 7 strikes {0.7..1.3} x L0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for sid in range(n_structures):
        N = int(rng.integers(8, 41))
        delta = float(rng.choice([0.25, 0.5]))
        L0 = rng.uniform(0.01, 0.06, size=N)
        alpha = float(rng.uniform(12.0, 25.0))
        beta = float(rng.uniform(-5.0, 0.0))
        dnig = float(rng.uniform(0.5, 1.5))
        s = int(round(delta / 0.025))
        out.append(make_structure(N, delta, L0, s, exp_decay_vol(),
                                  np.linspace(0.7, 1.3, 7), alpha=alpha, beta=beta,
                                  delta_nig=dnig, struct_id=sid,
                                  name=f"batched_{sid:02d}"))
    return out


# Euro zero-coupon bond prices on 19 Feb 2002 (paper Table 3.1), T = 0.5..5.
KLUGE_ZCB = np.array([0.9833630, 0.9647388, 0.9435826, 0.9228903, 0.9006922,
                      0.8790279, 0.8568412, 0.8352144, 0.8133497, 0.7920573])


def kluge_example(steps_per_period: int = 5, strike_mult=(0.8, 0.9, 1.0, 1.1, 1.2)
                  ) -> TermStructure:
    """The paper's numerical example (Section 4): T_i = i/2, i = 1..9, T_* = 5,
    forwards from the Table 3.1 bond prices via eq. (i-val), constant vols
    0.20, 0.19, ..., 0.12, NIG with alpha = delta = 1.5, beta = mu = 0."""
    B = KLUGE_ZCB
    N = 9
    delta = 0.5
    L0 = (B[:N] / B[1:N + 1] - 1.0) / delta
    vols = 0.20 - 0.01 * np.arange(N)
    return make_structure(N, delta, L0, steps_per_period,
                          lambda t, T, r: float(vols[r]), list(strike_mult),
                          alpha=1.5, beta=0.0, delta_nig=1.5, B0_T1=float(B[0]),
                          name="kluge_n9")


def swap_rates(ts: TermStructure) -> np.ndarray:
    """Forward co-terminal swap rates S_r(0) = (B(0,T_{r+1}) - B(0,T_*)) /
    sum_{l>=r} delta_l B(0,T_{l+2}) from the initial forwards (bond prices by
    eq. (i-val))."""
    P = ts.B0_T1 / np.concatenate([[1.0], np.cumprod(1.0 + ts.delta * ts.L0)])  # B(0,T_1..T_*)
    ann = np.cumsum((ts.delta * P[1:])[::-1])[::-1]
    return (P[:-1] - P[-1]) / ann


def coterminal_swaptions(ts: TermStructure, strike_mult=(0.8, 1.0, 1.2)) -> TermStructure:
    """The same model pricing payer swaptions instead of caplets: expiry at
    each fixing date T_{r+1}, underlying swap over the accrual periods r..N-1
    (to T_*), strikes strike_mult x the forward swap rate."""
    mult = np.atleast_1d(np.asarray(strike_mult, dtype=np.float64))
    out = ts.copy(strikes=swap_rates(ts)[:, None] * mult[None, :])
    out.product = 1
    out.name = ts.name + "_swaptions"
    out.validate_shapes()
    return out


def brownian(N: int = 6, delta: float = 0.5, L0=0.05, vol=0.2, c: float = 1.0,
             steps_per_period: int = 20, strike_mult=(0.9, 1.0, 1.1)) -> TermStructure:
    """Brownian special case (c > 0, no jumps) for the Black-formula check."""
    return make_structure(N, delta, L0, steps_per_period, lambda t, T, r: vol,
                          list(strike_mult), driver=DRIVER_BROWNIAN, c=c,
                          name=f"brownian_n{N}")


WORKLOADS = {
    "plain_n10": plain_fp64,
    "gpu_n20": gpu_scale,
    "mlp_n40": learned_drift,
    "adjoint_n40": adjoint_greeks,
    "kluge_n9": kluge_example,
    "mp_n60": maturity_parallel,
}
