"""Pins of the oracle's drift against the mathematics, not against itself.

The drift of eq. (LIBOR-drift-PT) (paper Section 2) for the pure-jump NIG
driver is  b_i = -A_i,  A_i = int [(e^{lambda_i x} - 1) prod_{l>i} beta_l(x)
- lambda_i x] F(dx).  The oracle evaluates kappa in closed form and the rest
with a 64-node rule.  Pinned here:

* the NIG cumulant and Lévy density against arbitrary-precision quadrature
  and Bessel functions (mpmath);
* the 64-node rule against the closed-form second moment of the Lévy measure;
* the whole drift against the exact subset expansion of the product
  (Section 3.2, eq. (product)): writing beta_l = (1 - ell_l) + ell_l e^{lambda_l x},
  A_i = sum_U p_U [kappa(lambda_i + lambda_U) - kappa(lambda_U)] over subsets U
  of the later rates, p_U = prod_{l in U} ell_l prod_{l not in U}(1 - ell_l);
* for N = 40, where 2^39 subsets are too many, against adaptive mpmath
  quadrature of the coupling integrand;
* the first-order expansion A' (eq. (drifta)) is O(ell^2) and the second-order
  A'' (eq. (drifta2)) with its first-order bracket written -kappa(l_i) -
  kappa(l_l) is O(ell^3) from the oracle's drift; the bracket as printed,
  +kappa(l_i) + kappa(l_l), is only O(ell) accurate (a sign misprint).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import workloads
from oracle import rule


def kappa_nig(u, alpha, beta, delta):
    """Closed-form NIG cumulant of the compensated driver (log E e^{u H_1})."""
    gamma = math.sqrt(alpha**2 - beta**2)
    mu = -delta * beta / gamma
    u = np.asarray(u, dtype=np.float64)
    return mu * u + delta * (gamma - np.sqrt(alpha**2 - (beta + u) ** 2))


def _levy_density_mp(x, alpha, beta, delta):
    x = mp.mpf(x)
    return delta * alpha / mp.pi * mp.exp(beta * x) * mp.besselk(1, alpha * abs(x)) / abs(x)


def _expm1_minus_linear(ux):
    """e^{ux} - 1 - ux without cancellation near 0 (Taylor series below 0.01)."""
    if abs(ux) < mp.mpf("0.01"):
        return mp.fsum(ux**n / mp.factorial(n) for n in range(2, 14))
    return mp.expm1(ux) - ux


def test_levy_density_vs_mpmath():
    mp.mp.dps = 30
    for (a, b, d) in [(18.0, -4.0, 1.0), (1.5, 0.0, 1.5), (12.3, -0.7, 0.6)]:
        for x in [1e-7, -3e-5, 0.01, -0.2, 0.9, 2.5, -7.0, 20.0]:
            ref = float(_levy_density_mp(x, a, b, d))
            got = float(rule.nig_levy_density(np.array([x]), a, b, d)[0])
            assert abs(got / ref - 1.0) < 1e-13, (a, b, d, x, got, ref)


def test_kappa_table_vs_levy_integral(oracle_mod):
    """kappa(u) = int (e^{ux} - 1 - ux) F(dx) (eq. (cumulant)) by mpmath quadrature."""
    mp.mp.dps = 25
    us = [-2.0, -0.5, 0.15, 1.0, 3.0, 5.0]
    ts = workloads.make_structure(len(us), 0.5, 0.03, 2, lambda t, T, r: us[r], [1.0])
    o = oracle_mod.Oracle(ts)
    for r, u in enumerate(us):
        f = lambda x: _expm1_minus_linear(u * x) * _levy_density_mp(x, ts.alpha, ts.beta,
                                                                     ts.delta_nig)
        ref = float(mp.quad(f, [-mp.inf, -1, 0]) + mp.quad(f, [0, 1, mp.inf]))
        # the closed form subtracts terms of size |mu u| + delta (gamma + sqrt(...)):
        # allow a few FP64 ulps of those, relative to the (much smaller) result
        gamma = math.sqrt(ts.alpha**2 - ts.beta**2)
        sq = math.sqrt(ts.alpha**2 - (ts.beta + u) ** 2)
        scale = abs(ts.delta_nig * ts.beta / gamma * u) + ts.delta_nig * (gamma + sq)
        tol = 8 * 2.0**-53 * scale + 1e-15 * abs(ref)
        assert abs(o.kappa[0, r] - ref) < tol, (u, o.kappa[0, r], ref, tol)


@pytest.mark.parametrize("wl", ["plain_n10", "gpu_n20", "mlp_n40", "kluge_n9"])
def test_rule_second_moment(wl):
    """sum_q W_q x_q^2 = int x^2 F(dx) = Var H_1 = delta alpha^2 / gamma^3."""
    ts = workloads.WORKLOADS[wl]()
    x, W, _ = rule.quadrature_rule(ts.alpha, ts.beta, ts.delta_nig, ts.vol, ts.tenor,
                                   ts.steps_per_period)
    gamma = math.sqrt(ts.alpha**2 - ts.beta**2)
    var = ts.delta_nig * ts.alpha**2 / gamma**3
    assert len(x) == 64 and np.all(W > 0)
    assert abs(np.sum(W * x * x) / var - 1.0) < 1e-9


def _subset_A(lam_i, lam_later, ell_later, kap):
    """Exact A_i = sum over subsets U of later rates of p_U [kappa(l_i + l_U) - kappa(l_U)]."""
    p = np.array([1.0])
    lu = np.array([0.0])
    for lam_l, ell_l in zip(lam_later, ell_later):
        p = np.concatenate([p * (1.0 - ell_l), p * ell_l])
        lu = np.concatenate([lu, lu + lam_l])
    terms = p * (kap(lam_i + lu) - kap(lu))
    return math.fsum(terms.tolist())


@pytest.mark.parametrize("wl,steps", [("plain_n10", [0, 37, 95]), ("gpu_n20", [0, 150]),
                                      ("kluge_n9", [0, 22])])
def test_drift_vs_exact_subset_expansion(oracle_mod, wl, steps):
    ts = workloads.WORKLOADS[wl]()
    o = oracle_mod.Oracle(ts)
    kap = lambda u: kappa_nig(u, ts.alpha, ts.beta, ts.delta_nig)
    rng = np.random.default_rng(3)
    for k in steps:
        first = k // ts.steps_per_period
        for L in (ts.L0, ts.L0 * np.exp(rng.normal(0.0, 0.3, ts.n_rates))):
            b = o.drift(k, L)
            lam = ts.vol[k]
            ell = ts.delta * L / (1.0 + ts.delta * L)
            for i in range(first, ts.n_rates):
                A = _subset_A(lam[i], lam[i + 1:], ell[i + 1:], kap)
                assert abs(-b[i] - A) <= 1e-11 * abs(A), (wl, k, i, -b[i], A)
                # the coupling part alone (A minus kappa(lambda_i))
                coup_ref = A - float(kap(lam[i]))
                coup = -b[i] - o.kappa[k, i]
                if i < ts.n_rates - 1:
                    assert abs(coup - coup_ref) <= 2e-10 * abs(coup_ref), (wl, k, i, coup, coup_ref)
                else:
                    assert coup == 0.0


@pytest.mark.slow
def test_drift_n40_vs_adaptive_quadrature(oracle_mod):
    """N = 40: the coupling integral against adaptive quadrature of the integrand."""
    mp.mp.dps = 20
    ts = workloads.learned_drift()
    o = oracle_mod.Oracle(ts)
    k = 0
    L = ts.L0
    b = o.drift(k, L)
    lam = ts.vol[k]
    ell = ts.delta * L / (1.0 + ts.delta * L)
    for i in (0, 17, 38):
        def f(x):
            # prod_l beta_l(x) - 1 as expm1(sum log1p(.)), accurate near x = 0
            logprod = mp.fsum(mp.log1p(ell[l] * mp.expm1(lam[l] * x))
                              for l in range(i + 1, ts.n_rates))
            return (mp.expm1(lam[i] * x) * mp.expm1(logprod)
                    * _levy_density_mp(x, ts.alpha, ts.beta, ts.delta_nig))
        ref = float(mp.quad(f, [-mp.inf, -1, 0]) + mp.quad(f, [0, 1, mp.inf]))
        coup = -b[i] - o.kappa[k, i]
        assert abs(coup / ref - 1.0) < 1e-9, (i, coup, ref)


def _expansions(lam, ell, i, kap):
    """A' (eq. (drifta)), A'' with the corrected and with the printed first-order bracket."""
    li = lam[i]
    first = 0.0
    first_printed = 0.0
    for l in range(i + 1, len(lam)):
        first += ell[l] * (kap(li + lam[l]) - kap(li) - kap(lam[l]))
        first_printed += ell[l] * (kap(li + lam[l]) + kap(li) + kap(lam[l]))
    second = 0.0
    for k in range(i + 1, len(lam)):
        for l in range(k + 1, len(lam)):
            second += ell[l] * ell[k] * (kap(li + lam[l] + lam[k]) - kap(li + lam[l])
                                         - kap(li + lam[k]) - kap(lam[k] + lam[l])
                                         + kap(li) + kap(lam[l]) + kap(lam[k]))
    a1 = kap(li) + first
    return a1, a1 + second, kap(li) + first_printed + second


def test_drift_expansion_orders(oracle_mod):
    ts = workloads.plain_fp64()
    o = oracle_mod.Oracle(ts)
    kap = lambda u: float(kappa_nig(u, ts.alpha, ts.beta, ts.delta_nig))
    k, i = 0, 0
    lam = ts.vol[k]
    errs = []
    for eps in (1.0, 0.5, 0.25):
        L = ts.L0 * eps
        A = -o.drift(k, L)[i]
        ell = ts.delta * L / (1.0 + ts.delta * L)
        a1, a2, a2_printed = _expansions(lam, ell, i, kap)
        errs.append((abs(A - a1), abs(A - a2), abs(A - a2_printed)))
    e = np.array(errs)
    # halving ell divides the A' error by ~4 and the corrected A'' error by ~8
    assert 3.2 < e[0, 0] / e[1, 0] < 4.8 and 3.2 < e[1, 0] / e[2, 0] < 4.8
    assert 6.0 < e[0, 1] / e[1, 1] < 10.0 and 6.0 < e[1, 1] / e[2, 1] < 10.0
    # the printed sign leaves an O(ell) error, far larger than A''
    assert 1.6 < e[0, 2] / e[1, 2] < 2.4
    assert e[0, 2] > 1e3 * e[0, 1]


def test_first_order_drift_of_the_oracle(oracle_mod):
    """The oracle's first-order drift (eq. (drifta)) is the A' of the test above
    (an independent transcription), its error against the product-form drift
    shrinks 4x when the forwards halve, and at N = 40 it agrees with the
    surrogate reference's first-order coupling."""
    from oracle import mlp as M
    ts = workloads.plain_fp64()
    o = oracle_mod.Oracle(ts)
    kap = lambda u: float(kappa_nig(u, ts.alpha, ts.beta, ts.delta_nig))
    errs = []
    for eps in (1.0, 0.5, 0.25):
        L = ts.L0 * eps
        b1 = o.drift(0, L, order=1)
        ell = ts.delta * L / (1.0 + ts.delta * L)
        a1, _, _ = _expansions(ts.vol[0], ell, 0, kap)
        assert abs(-b1[0] - a1) <= 1e-14 * abs(a1)
        errs.append(abs(b1[0] - o.drift(0, L)[0]))
    assert 3.2 < errs[0] / errs[1] < 4.8 and 3.2 < errs[1] / errs[2] < 4.8
    t40 = workloads.learned_drift()
    o40 = oracle_mod.Oracle(t40)
    k = 137
    m = k // t40.steps_per_period
    L = t40.L0 * np.exp(np.linspace(-0.2, 0.3, 40))
    b1 = o40.drift(k, L, order=1)
    ell = t40.delta * L / (1.0 + t40.delta * L)
    ell[:m] = 0.0
    C1 = M.first_order_coupling(ell[None, :], np.asarray(t40.vol[k]), t40)[0]
    assert np.allclose(-b1[m:] - o40.kappa[k, m:], C1[m:], rtol=1e-12, atol=1e-18)


def test_first_order_scheme_is_exact_for_brownian_driver(oracle_mod):
    """With a Brownian driver the coupling c lambda_i sum ell_l lambda_l is linear
    in ell, so the first-order scheme reproduces the full scheme."""
    ts = workloads.brownian()
    o = oracle_mod.Oracle(ts)
    L = ts.L0 * 1.3
    for k in (0, 25, 100):
        assert np.allclose(o.drift(k, L, order=1), o.drift(k, L), rtol=1e-14,
                           atol=0, equal_nan=True)
    a = o.price(3, 500)
    b = o.price(0, 500)
    assert np.allclose(a["price"], b["price"], rtol=1e-12, atol=0)


def test_second_order_drift_of_the_oracle(oracle_mod):
    """The oracle's second-order drift (eq. (drifta2) with the corrected sign)
    is the A'' of the independent transcription above, its error against the
    product-form drift shrinks 8x when the forwards halve, and for a Brownian
    driver (quadratic cumulant: every third difference vanishes) it is exact."""
    ts = workloads.plain_fp64()
    o = oracle_mod.Oracle(ts)
    kap = lambda u: float(kappa_nig(u, ts.alpha, ts.beta, ts.delta_nig))
    errs = []
    for eps in (1.0, 0.5, 0.25):
        L = ts.L0 * eps
        b2 = o.drift(0, L, order=2)
        ell = ts.delta * L / (1.0 + ts.delta * L)
        _, a2, _ = _expansions(ts.vol[0], ell, 0, kap)
        assert abs(-b2[0] - a2) <= 1e-14 * abs(a2)
        errs.append(abs(b2[0] - o.drift(0, L)[0]))
    assert 6.0 < errs[0] / errs[1] < 10.0 and 6.0 < errs[1] / errs[2] < 10.0
    tb = workloads.brownian()
    ob = oracle_mod.Oracle(tb)
    L = tb.L0 * 1.3
    assert np.allclose(ob.drift(40, L, order=2), ob.drift(40, L), rtol=1e-14, atol=0,
                       equal_nan=True)
