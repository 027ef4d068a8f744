"""The learned drift surrogate on the GPU: its BF16-MFMA forward and backward
kernels against the FP64 reference (oracle/mlp.py, with the device's BF16
operand rounding reproduced), its training labels against the FP64 oracle's
drift, training progress, and what the trained network gains over the
first-order expansion it corrects, judged against the quadrature drift.

Tolerances: the device accumulates BF16 products in FP32 and evaluates the
activation with hardware exp / reciprocal (relative error ~1e-6); the
reference accumulates exactly.  An activation that lands within that error of
a BF16 rounding boundary rounds the other way (one BF16 ulp, 2^-8 relative),
so outputs agree to ~1e-3 of their scale and gradients, which sum many such
products, to ~1e-2 in norm.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import mlp as M

pytestmark = pytest.mark.gpu

FULL, PICARD = 0, 1


def _features(rng, n, N=40):
    f = np.zeros((n, 96), dtype=np.float32)
    i = rng.integers(0, N, n)
    f[:, 0] = rng.uniform(0, 1, n)
    for j in range(n):
        f[j, 1 + i[j] + 1:1 + N] = rng.normal(0, 0.3, N - i[j] - 1)
        f[j, 41 + i[j]] = 1.0
    return f


def test_forward_and_gradients_match_reference(gpu_lib):
    rng = np.random.default_rng(1)
    with gpu_lib.Mlp(seed=7) as net:
        p = net.params().astype(np.float64)
        # non-zero biases exercise every parameter
        p[6144:6208] = rng.normal(0, 0.1, 64)
        p[10304:10368] = rng.normal(0, 0.1, 64)
        p[14464:14528] = rng.normal(0, 0.1, 64)
        p[14592] = 0.05
        net.set_params(p.astype(np.float32))
        p = net.params().astype(np.float64)
        X = _features(rng, 1000)
        t = rng.normal(0, 1, 1000).astype(np.float32)
        out = net.eval(X, t)
    y_ref, _ = M.forward(p, X, bf=True)
    scale = np.sqrt(np.mean(y_ref ** 2))
    assert np.max(np.abs(out["y"] - y_ref)) <= 2e-3 * scale + 1e-6
    loss_ref, g_ref = M.loss_and_grad(p, X, t, bf=True)
    assert abs(out["loss"] - loss_ref) <= 1e-3 * loss_ref
    offs = [0, 6144, 6208, 10304, 10368, 14464, 14528, 14592, 14593]
    for a, b in zip(offs[:-1], offs[1:]):
        ga, gr = out["grad"][a:b], g_ref[a:b]
        err = np.linalg.norm(ga - gr) / max(np.linalg.norm(gr), 1e-30)
        assert err < 1e-2, (a, b, err)
    # without the BF16 rounding the reference differs by more than the device does
    y64, _ = M.forward(p, X, bf=False)
    assert np.max(np.abs(out["y"] - y_ref)) < np.max(np.abs(y64 - y_ref)) + 1e-6


def _kappa(u, ts):
    g = math.sqrt(ts.alpha ** 2 - ts.beta ** 2)
    mu = -ts.delta_nig * ts.beta / g
    return mu * u + ts.delta_nig * (g - np.sqrt(ts.alpha ** 2 - (ts.beta + u) ** 2))


def test_training_labels_match_oracle(gpu_lib, oracle_mod):
    ts = workloads.learned_drift()
    o = oracle_mod.Oracle(ts)
    with gpu_lib.Plan(ts, precision=0, max_paths=1024) as plan, gpu_lib.Mlp(seed=1) as net:
        n_pairs = net.generate(plan, 256, 8, seed=5)
        info = net.info()
        assert n_pairs == info["n_pairs"] > 0 and info["sigma"] > 0
        rng = np.random.default_rng(3)
        d = net.pairs(rng.choice(n_pairs, 60, replace=False))
    s = ts.steps_per_period
    for j in range(60):
        k, i, X = int(d["k"][j]), int(d["rate"][j]), d["state"][j].astype(np.float64)
        first = k // s
        assert first <= i < ts.n_rates
        L = ts.L0 * np.exp(X)
        C = -o.drift(k, L)[i] - o.kappa[k, i]
        ell = ts.delta * L / (1 + ts.delta * L)
        lam = ts.vol[k]
        C1 = sum(ell[l] * (_kappa(lam[i] + lam[l], ts) - _kappa(lam[i], ts) - _kappa(lam[l], ts))
                 for l in range(i + 1, ts.n_rates))
        assert abs(d["label"][j] - (C - C1)) <= 1e-6 * abs(C) + 1e-12, (j, d["label"][j], C - C1)
        f = d["feat"][j]
        T = np.concatenate([[0.0], ts.tenor])
        tk = T[first] + (k - first * s) * (T[first + 1] - T[first]) / s
        assert f[0] == M.bf16(tk / ts.tenor[-1])
        assert np.array_equal(f[1:1 + i + 1], np.zeros(i + 1))
        assert np.array_equal(f[1 + i + 1:41], M.bf16(X[i + 1:]))
        assert f[41 + i] == 1.0 and np.sum(f[41:]) == 1.0
    # the trust box holds every recorded state of a live rate
    assert np.all(info["lo"] <= 0.0) and np.all(info["hi"][:-1] >= 0.0)


def test_training_reduces_loss(gpu_lib):
    ts = workloads.learned_drift()
    with gpu_lib.Plan(ts, precision=0, max_paths=1024) as plan, gpu_lib.Mlp(seed=1) as net:
        net.generate(plan, 2048, 16, seed=2)
        loss = net.train(400, batch=4096, lr=2e-3, seed=3)
    assert np.all(np.isfinite(loss))
    assert loss[-40:].mean() < 0.1 * loss[:10].mean(), (loss[:10].mean(), loss[-40:].mean())


@pytest.fixture(scope="module")
def trained(gpu_lib):
    """The N=40 quarterly workload's surrogate, trained on ~2^22 quadrature pairs
    (the benchmark's datagen and training configuration)."""
    ts = workloads.learned_drift()
    plan = gpu_lib.Plan(ts, precision=0, max_paths=1 << 20)
    net = gpu_lib.Mlp(seed=1)
    n_pairs = net.generate(plan, 12800, 16, seed=1)
    loss = net.train(3000, batch=16384, lr=2e-3, seed=1)
    yield ts, plan, net, n_pairs, loss
    net.close()
    plan.close()


def _surrogate_oracle(oracle_mod, ts, net, paths, use_net=True):
    o = oracle_mod.Oracle(ts)
    info = net.info()
    return M.surrogate_paths(o, net.params().astype(np.float64), info["lo"], info["hi"],
                             info["sigma"], paths, use_net=use_net)


@pytest.mark.parametrize("use_net", [True, False])
def test_surrogate_paths_match_oracle(gpu_lib, oracle_mod, trained, use_net):
    """Per-path fixings of the surrogate scheme (and of the first-order scheme)
    against the FP64 oracle of the same scheme with the same weights, box and
    streams: the FP32 path tolerance of the FULL scheme (2e-5 relative)."""
    import torch
    ts, plan, net, _, _ = trained
    n = 128
    fix = torch.empty((n, 2 * ts.n_rates), dtype=torch.float64, device="cuda")
    plan.execute_mlp(net if use_net else None, use_net, n, seed=1, judge_stride=1, path_fix=fix)
    torch.cuda.synchronize()
    f = fix.cpu().numpy()
    sums, Lo, Do = _surrogate_oracle(oracle_mod, ts, net, np.arange(n), use_net)
    assert np.all(np.abs(f[:, 0::2] / Lo - 1.0) < 2e-5)
    assert np.all(np.abs(f[:, 1::2] / Do - 1.0) < 2e-5)
    ref = oracle_mod.finish(sums, ts.delta, ts.L0, ts.B0_T1 / np.prod(1.0 + ts.delta * ts.L0))
    got = plan.results()
    live = ref["price"] > 0
    assert np.all(np.abs(got["price"][live] / ref["price"][live] - 1.0) < 1e-4)
    st = plan.mlp_stats()
    assert st["rate_steps"] == n * sum(ts.n_rates - k // ts.steps_per_period
                                       for k in range(ts.n_steps))
    if not use_net:
        assert st["fallbacks"] == 0


def test_surrogate_full_size_sampled_paths(gpu_lib, oracle_mod, trained):
    """The benchmark launch (2^20 paths): sampled per-path fixings against the
    oracle of the surrogate scheme."""
    import torch
    ts, plan, net, _, _ = trained
    n = 1 << 20
    fix = torch.empty((n, 2 * ts.n_rates), dtype=torch.float64, device="cuda")
    plan.execute_mlp(net, True, n, seed=1, path_fix=fix)
    torch.cuda.synchronize()
    f = fix.cpu().numpy()
    sample = np.array([0, 4095, 77777, 524288, n - 1])
    _, Lo, Do = _surrogate_oracle(oracle_mod, ts, net, sample)
    assert np.all(np.abs(f[sample, 0::2] / Lo - 1.0) < 2e-5)
    assert np.all(np.abs(f[sample, 1::2] / Do - 1.0) < 2e-5)


def test_empty_trust_box_is_full_euler(gpu_lib, trained):
    """An empty trust box sends every coupling to the quadrature: the surrogate
    pass must then reproduce the FULL pass bit for bit."""
    ts, plan, net, _, _ = trained
    n = 1 << 14
    info = net.info()
    plan.execute(FULL, n, seed=3)
    full = plan.results()
    try:
        net.set_box(np.ones(40), -np.ones(40))
        plan.execute_mlp(net, True, n, seed=3)
        got = plan.results()
        st = plan.mlp_stats()
    finally:
        net.set_box(info["lo"], info["hi"])
    assert np.array_equal(got["price"], full["price"])
    assert np.array_equal(got["mart_resid"], full["mart_resid"])
    # every coupled rate-step fell back; the last rate has no coupling
    s = ts.steps_per_period
    coupled = n * sum(ts.n_rates - 1 - k // s for k in range(ts.n_steps) if k // s < ts.n_rates - 1)
    assert st["fallbacks"] == coupled
    with pytest.raises(gpu_lib.LLLError):
        net.set_box(np.full(40, np.nan), np.ones(40))


def test_first_order_scheme_matches_surrogate_kernel_without_network(gpu_lib, trained):
    """The path kernel's first-order scheme and the surrogate kernel without its
    network evaluate the same drift (eq. (drifta)) on the same streams, in FP32
    with different summation orders."""
    ts, plan, _, _, _ = trained
    n = 1 << 14
    plan.execute(3, n, seed=2)
    a = plan.results()
    plan.execute_mlp(None, False, n, seed=2)
    b = plan.results()
    live = a["price"] > 0
    assert np.all(np.abs(b["price"][live] / a["price"][live] - 1.0) < 1e-6)
    assert np.array_equal(a["n_itm"], b["n_itm"])


def test_surrogate_gain_over_first_order(gpu_lib, trained):
    """Prices on common random numbers at the benchmark size (2^20 paths): the
    surrogate against the FULL quadrature drift, next to the first-order
    expansion alone, Picard and the frozen drift."""
    ts, plan, net, n_pairs, loss = trained
    n = 1 << 20
    assert n_pairs >= 4_000_000
    res = {}
    plan.execute(FULL, n, seed=1)
    res["full"] = plan.results()["price"]
    plan.execute(PICARD, n, seed=1)
    res["picard"] = plan.results()["price"]
    plan.execute(2, n, seed=1)
    res["frozen"] = plan.results()["price"]
    plan.execute_mlp(None, False, n, seed=1)
    res["first_order"] = plan.results()["price"]
    plan.execute_mlp(net, True, n, seed=1, judge_stride=8)
    res["mlp"] = plan.results()["price"]
    stats = plan.mlp_stats()
    # caplets fixed at t = 0 have a deterministic payoff; out of the money it is 0
    live = res["full"] > 0.0
    for v in res.values():
        assert np.array_equal(v[~live], res["full"][~live])
    err = {k: np.max(np.abs(v[live] / res["full"][live] - 1.0)) for k, v in res.items()}
    print("max relative price error vs FULL:", {k: f"{v:.2e}" for k, v in err.items()})
    print("judge:", stats, "final loss", float(loss[-50:].mean()))
    assert err["mlp"] <= 1e-4
    assert err["mlp"] < err["first_order"]
    assert err["frozen"] > err["mlp"]
    assert stats["fallbacks"] <= 1e-3 * stats["rate_steps"]
    assert stats["judged"] > 0
    assert stats["judge_abs_err"] / stats["judge_abs_quad"] < 1e-4
