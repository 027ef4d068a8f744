"""Pins of the oracle's random-number pieces against things other than itself.

* Philox-4x32-10 words against AMD rocRAND's own engine (a separate
  implementation of Salmon et al. 2011), compiled host-only from its header.
* The 24-bit uniform map against exact integer arithmetic.
* The inverse-Gaussian subordinator and the NIG increment (the paper draws NIG
  numbers by the standard subordinator + normal mixture method, Section 4)
  against scipy's invgauss / norminvgauss distributions (KS) and the closed
  form moments of NIG(alpha, beta, delta dt, mu dt).
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import workloads

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_ref.cpp")


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rr") / "rr_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, HELPER], check=True)

    def run(cases):
        inp = "\n".join(" ".join("%08x" % v for v in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return [tuple(int(t, 16) for t in line.split()) for line in out.strip().splitlines()]
    return run


def test_philox_matches_rocrand(oracle_mod, rocrand_ref):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 0, 0, 0, 1, 0), (0, 1, 0, 0, 0, 0),
             (0, 0, 1, 0, 0, 0), (0, 0, 0, 1, 0, 0), (0, 0, 0, 0, 0, 1)]
    cases += [tuple(int(v) for v in rng.integers(0, 2**32, size=6)) for _ in range(200)]
    # the layout the method uses: counter (step, path_lo, path_hi, stream), key = seed 1
    cases += [(k, p, 0, 5, 1, 0) for k in (0, 1, 399) for p in (0, 1, 12345, 2**20 - 1)]
    ref = rocrand_ref(cases)
    for c, r in zip(cases, ref):
        got = tuple(int(w) for w in oracle_mod.philox4x32_10(c[:4], c[4:]))
        assert got == r, (c, got, r)


def test_uniform_map_exact(oracle_mod):
    # ((w >> 8) + 1/2) 2^-24: open interval (0, 1), exact in FP64 (25 significant
    # bits, so not in FP32: the increments are drawn in FP64 on both sides)
    assert oracle_mod.uniform(0) == 0.5 * 2.0**-24
    assert oracle_mod.uniform(0xFFFFFFFF) == 1.0 - 0.5 * 2.0**-24
    assert oracle_mod.uniform(0x00000100) == 1.5 * 2.0**-24
    for w in (0x12345678, 0x80000000, 0xDEADBEEF):
        u = oracle_mod.uniform(w)
        assert u == ((w >> 8) + 0.5) / 2**24
        assert 0.0 < u < 1.0


def _cdf_from_pdf(law, samples):
    """CDF of a continuous law by cumulative integration of its closed-form pdf on
    a fine grid (scipy's own norminvgauss.cdf integrates per point and is slow)."""
    sd = law.std()
    lo = samples.min() - sd
    hi = samples.max() + sd
    grid = np.linspace(lo, hi, 400001)
    pdf = law.pdf(grid)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf += law.cdf(lo)
    return lambda x: np.interp(x, grid, cdf)


def _nig_params(ts, dt):
    gamma = math.sqrt(ts.alpha**2 - ts.beta**2)
    mu_H = -ts.delta_nig * ts.beta / gamma
    return gamma, mu_H


@pytest.mark.parametrize("wl", ["plain_n10", "gpu_n20", "kluge_n9"])
def test_inverse_gaussian_ks(oracle_mod, wl):
    ts = workloads.WORKLOADS[wl]()
    o = oracle_mod.Oracle(ts, seed=11)
    k = 3
    dt = o.dt[k]
    gamma, _ = _nig_params(ts, dt)
    m = ts.delta_nig * dt / gamma          # IG mean
    lam = (ts.delta_nig * dt) ** 2          # IG shape
    V, _ = o.increments(k, 0, 200000)
    # IG(mean m, shape lam) == scipy invgauss(mu = m / lam, scale = lam)
    ks = stats.kstest(V, stats.invgauss(m / lam, scale=lam).cdf)
    assert ks.pvalue > 1e-3, ks
    assert abs(V.mean() - m) < 5 * math.sqrt(m**3 / lam / len(V))
    assert abs(V.var() / (m**3 / lam) - 1.0) < 0.05


@pytest.mark.parametrize("wl", ["plain_n10", "gpu_n20", "kluge_n9"])
def test_nig_increment_law(oracle_mod, wl):
    ts = workloads.WORKLOADS[wl]()
    o = oracle_mod.Oracle(ts, seed=5)
    k = 7
    dt = o.dt[k]
    gamma, mu_H = _nig_params(ts, dt)
    _, dH = o.increments(k, 1000, 200000)
    d = ts.delta_nig * dt
    law = stats.norminvgauss(ts.alpha * d, ts.beta * d, loc=mu_H * dt, scale=d)
    ks = stats.kstest(dH, _cdf_from_pdf(law, dH))
    assert ks.pvalue > 1e-3, ks
    # closed-form moments of NIG(alpha, beta, delta dt, mu_H dt): mean 0 (martingale),
    # variance delta dt alpha^2 / gamma^3
    var = d * ts.alpha**2 / gamma**3
    assert abs(dH.mean()) < 5 * math.sqrt(var / len(dH))
    assert abs(dH.var() / var - 1.0) < 0.05
    assert abs(law.mean()) < 1e-15 and abs(law.var() / var - 1) < 1e-10


def test_brownian_increment_law(oracle_mod):
    ts = workloads.brownian(N=4, c=0.7)
    o = oracle_mod.Oracle(ts, seed=2)
    k = 2
    V, dH = o.increments(k, 0, 200000)
    assert np.all(V == 0.0)
    sd = math.sqrt(ts.c * o.dt[k])
    ks = stats.kstest(dH / sd, stats.norm.cdf)
    assert ks.pvalue > 1e-3, ks


def test_increments_are_counter_based(oracle_mod):
    """Same (seed, step, path) gives the same draw; neighbouring counters differ."""
    ts = workloads.plain_fp64()
    a = oracle_mod.Oracle(ts, seed=1)
    b = oracle_mod.Oracle(ts, seed=1)
    c = oracle_mod.Oracle(ts, seed=2)
    _, x = a.increments(4, 100, 64)
    _, y = b.increments(4, 100, 64)
    _, z = c.increments(4, 100, 64)
    assert np.array_equal(x, y)
    assert not np.any(x == z)
    assert a.increment(4, 100)[1] == x[0]
