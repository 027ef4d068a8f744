"""Quadrature rule over the NIG Lévy measure, FP64, for the CPU oracle.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use anything under ``oracle/``; the
product path never does.

What is computed (paper Section 2, eq. (LIBOR-drift-PT); Section 4 for the
NIG driver):

* the jump part of the drift contains an integral over the Lévy measure F of
  the driver.  Its linear-in-``x`` compensated part equals the cumulant
  kappa(lambda_i) (eq. (cumulant)) and is evaluated in closed form; the rest,
  the coupling integral  int (e^{lambda_i x} - 1)(prod_l beta_l(x) - 1) F(dx),
  is evaluated with a fixed 64-node rule;
* the rule: 32-point Gauss-Legendre nodes v_j, weights w_j on [0, 1]; on each
  side of the origin the substitution x = +-X_pm v^2 (dx = 2 X_pm v dv), so
  the nodes are x = +X_+ v_j^2 (q = 0..31) and x = -X_- v_j^2 (q = 32..63)
  with weights W = w_j 2 X_pm v_j f(x);
* the truncation points: the integrand decays like e^{-(alpha - beta - Lambda_+) x}
  on the right and e^{-(alpha + beta - Lambda_-)|x|} on the left, where
  Lambda_+ (Lambda_-) is the largest sum over live rates of the positive
  (negative) vols at any step; X_pm = min(36 / decay rate, 40), i.e. the tail
  beyond is below e^{-36};
* f is the NIG Lévy density  f(x) = (delta alpha / pi) e^{beta x} K_1(alpha |x|) / |x|.

Library primitives used as steps: ``numpy.polynomial.legendre.leggauss`` for
the Gauss-Legendre rule and ``scipy.special.k1e`` (exponentially scaled
modified Bessel function of the second kind, order 1).
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.special import k1e

N_GL = 32
N_NODES = 2 * N_GL
TAIL_EXPONENT = 36.0
X_CAP = 40.0


def gauss_legendre_01(n: int = N_GL):
    """Gauss-Legendre nodes and weights on [0, 1]."""
    g, w = leggauss(n)
    return 0.5 * (g + 1.0), 0.5 * w


def nig_levy_density(x, alpha, beta, delta_nig):
    """NIG Lévy density (delta alpha/pi) e^{beta x} K_1(alpha|x|)/|x|, written with
    the scaled Bessel function so that large |x| does not overflow."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    return (delta_nig * alpha / math.pi) * np.exp(beta * x - alpha * ax) * k1e(alpha * ax) / ax


def live_vol_sums(vol: np.ndarray, tenor: np.ndarray, steps_per_period: int):
    """Lambda_+ and Lambda_-: max over steps of the sum over live rates of the
    positive (resp. negative) parts of lambda(t_k, T_i)."""
    N = len(tenor)
    lam_p = 0.0
    lam_m = 0.0
    for k in range(vol.shape[0]):
        m = k // steps_per_period          # period; live rates r >= m
        row = vol[k, m:N]
        lam_p = max(lam_p, float(np.sum(np.maximum(row, 0.0))))
        lam_m = max(lam_m, float(np.sum(np.maximum(-row, 0.0))))
    return lam_p, lam_m


def truncation(alpha, beta, lam_p, lam_m):
    """X_+ and X_- of the rule (see module docstring)."""
    right = alpha - beta - lam_p
    left = alpha + beta - lam_m
    if right <= 0.0 or left <= 0.0:
        raise ValueError("exponential-moment condition violated: drift integral diverges")
    return min(TAIL_EXPONENT / right, X_CAP), min(TAIL_EXPONENT / left, X_CAP)


def quadrature_rule(alpha, beta, delta_nig, vol, tenor, steps_per_period):
    """Nodes x_q and weights W_q (q = 0..63) of the coupling-integral rule."""
    lam_p, lam_m = live_vol_sums(vol, tenor, steps_per_period)
    xp, xm = truncation(alpha, beta, lam_p, lam_m)
    v, w = gauss_legendre_01()
    x = np.concatenate([xp * v * v, -xm * v * v])
    jac = np.concatenate([2.0 * xp * v * w, 2.0 * xm * v * w])
    W = jac * nig_levy_density(x, alpha, beta, delta_nig)
    return x, W, (xp, xm, lam_p, lam_m)
