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


def test_surrogate_and_picard_against_oracle_full(gpu_lib, oracle_mod, trained):
    """The metric's accuracy gate judged by the FP64 oracle: surrogate-drift
    and Picard prices at 2^16 paths against the oracle's FULL prices on the
    same streams (stored sums, tests/golden/oracle_sums_mlp_n40_2p16.json),
    per caplet-strike, with the near-zero floor of the parity tests."""
    from test_gpu_fullsize import C4_FILE, golden_sums, oracle_prices, per_caplet_errors, _table
    ts, plan, net, _, _ = trained
    n = 1 << 16
    ref = oracle_prices(oracle_mod, ts, golden_sums(C4_FILE, "full"))
    plan.execute_mlp(net, True, n, seed=1)
    mlp = plan.results()
    plan.execute_mlp(None, False, n, seed=1)
    first = plan.results()
    plan.execute(PICARD, n, seed=1)
    pic = plan.results()
    err = {}
    for name, got in (("mlp", mlp), ("picard", pic), ("first_order", first)):
        rel, floored = per_caplet_errors(got, ref, ts)
        _table(f"mlp_n40 {name} 2^16 paths vs FP64 oracle FULL", rel, floored)
        err[name] = float(rel.max())
    print("max per-caplet error vs oracle FULL:", {k: f"{v:.2e}" for k, v in err.items()})
    assert err["mlp"] <= 1e-4 and err["picard"] <= 1e-4
    assert err["mlp"] < err["first_order"]


def _kappa_np(u, ts):
    g = math.sqrt(ts.alpha ** 2 - ts.beta ** 2)
    return -ts.delta_nig * ts.beta / g * u + ts.delta_nig * (g - np.sqrt(ts.alpha ** 2 - (ts.beta + u) ** 2))


def test_surrogate_drift_judged_against_fp64_quadrature(gpu_lib, oracle_mod, trained):
    """The trained network's coupling C'_i + sigma net(features) against the
    FP64 oracle's quadrature coupling at states drawn on the host: step k and
    rate i uniform over the coupled (step, rate) pairs, log-rate states X_l
    normal with the mean and variance of the driver-only dynamics
    (-sum kappa(lambda) dt, sum lambda^2 Var(H_1) dt) up to t_k."""
    ts, plan, net, _, _ = trained
    o = oracle_mod.Oracle(ts)
    info = net.info()
    sigma = info["sigma"]
    N, s = ts.n_rates, ts.steps_per_period
    rng = np.random.default_rng(12)
    g = math.sqrt(ts.alpha ** 2 - ts.beta ** 2)
    var_h1 = ts.delta_nig * ts.alpha ** 2 / g ** 3
    T = np.concatenate([[0.0], ts.tenor])
    feats, labels, quads = [], [], []
    for _ in range(400):
        k = int(rng.integers(0, (N - 1) * s))
        m = k // s
        i = int(rng.integers(m, N - 1))
        mean = -np.sum(_kappa_np(ts.vol[:k], ts) * o.dt[:k, None], axis=0)
        var = np.sum(ts.vol[:k] ** 2 * o.dt[:k, None], axis=0) * var_h1
        X = mean + np.sqrt(var) * rng.normal(size=N)
        X[:m] = 0.0
        L = ts.L0 * np.exp(X)
        quad = -o.drift(k, L)[i] - o.kappa[k, i]
        ell = ts.delta * L / (1 + ts.delta * L)
        ell[:m] = 0.0
        c1 = M.first_order_coupling(ell[None, :], ts.vol[k], ts)[0, i]
        tk = T[m] + (k - m * s) * (T[m + 1] - T[m]) / s
        feats.append(M.features(float(np.float32(tk / T[N])), X[None, :], i)[0])
        labels.append(c1)
        quads.append(quad)
    y = net.eval(np.array(feats, dtype=np.float32))["y"].astype(np.float64)
    C = np.array(labels) + sigma * y
    q = np.array(quads)
    rel = np.abs(C - q) / np.abs(q)
    first = np.abs(np.array(labels) - q) / np.abs(q)
    print(f"surrogate coupling vs FP64 quadrature at 400 host states: mean |err| / mean |C| "
          f"{np.mean(np.abs(C - q)) / np.mean(np.abs(q)):.2e}, max rel {rel.max():.2e}; "
          f"first-order alone: {np.mean(np.abs(np.array(labels) - q)) / np.mean(np.abs(q)):.2e}, "
          f"max {first.max():.2e}")
    # the coupling enters the drift times dt; ~1e-3 of it is ~1e-6 of the price
    assert np.mean(np.abs(C - q)) / np.mean(np.abs(q)) < 1e-3
    assert np.mean(np.abs(C - q)) < 0.1 * np.mean(np.abs(np.array(labels) - q))


def test_training_update_matches_oracle(gpu_lib, oracle_mod):
    """Three Adam steps of lll_mlp_train_dev on pairs made on the host, from
    parameters set on the host, against the oracle's FP64 training loop (the
    same minibatches from its own Philox, the loss and gradient with the
    device's BF16 operand rounding, Adam with bias correction, the cosine
    learning rate).  The device accumulates in FP32 and evaluates GELU with
    hardware exp; a BF16 rounding flip moves one activation by 2^-8, so
    gradients agree to ~1e-2 in norm and individual entries can differ where
    the gradient is small.  Compared: the moments m, v per layer in norm, and
    the parameter moves element by element where the oracle's gradient is
    well above its own BF16-rounding sensitivity."""
    import torch
    rng = np.random.default_rng(21)
    p0 = rng.normal(0.0, 1.0, M.N_PARAMS) / np.sqrt(np.repeat(
        [96, 1, 64, 1, 64, 1, 64, 1], [6144, 64, 4096, 64, 4096, 64, 64, 1])) * 0.5
    p0 = p0.astype(np.float32).astype(np.float64)
    n_pairs, batch, steps, lr, seed, sigma = 3000, 256, 3, 1e-3, 5, 0.7
    feat = M.bf16(np.concatenate([rng.uniform(0, 1, (n_pairs, 1)),
                                  rng.normal(0, 0.3, (n_pairs, 40)),
                                  np.eye(40)[rng.integers(0, 40, n_pairs)],
                                  np.zeros((n_pairs, 15))], axis=1))
    labels = (np.tanh(feat[:, 1] - 0.5 * feat[:, 3]) + 0.2 * feat[:, 0]).astype(np.float32)
    with gpu_lib.Mlp(seed=1) as net:
        net.set_params(p0.astype(np.float32))
        fd = torch.tensor(feat.astype(np.float32)).to(torch.bfloat16).cuda()
        ld = torch.tensor(labels, dtype=torch.float32).cuda()
        loss_d = torch.zeros(steps, dtype=torch.float32, device="cuda")
        net.train_dev(fd, ld, sigma, steps, batch=batch, lr=lr, seed=seed, loss=loss_d)
        torch.cuda.synchronize()
        p_gpu = net.params().astype(np.float64)
        st = net.optimizer_state()
    assert st["step"] == steps
    p_ref, m_ref, v_ref, loss_ref = M.train(p0, feat, labels.astype(np.float64), sigma, steps,
                                            batch, lr, seed, oracle_mod.philox4x32_10)
    assert np.allclose(loss_d.cpu().numpy(), loss_ref, rtol=2e-3)
    # sensitivity of the oracle's gradient to the BF16 rounding: the last
    # step's gradient with and without the operand rounding
    idx = M.minibatch(oracle_mod.philox4x32_10, seed, steps, batch, n_pairs)
    _, g_bf = M.loss_and_grad(p_ref, feat[idx], labels[idx] / sigma, bf=True)
    _, g_64 = M.loss_and_grad(p_ref, feat[idx], labels[idx] / sigma, bf=False)
    offs = [0, 6144, 6208, 10304, 10368, 14464, 14528, 14592, 14593]
    for a, b in zip(offs[:-1], offs[1:]):
        for got, ref, tol in ((st["m"][a:b], m_ref[a:b], 2e-2), (st["v"][a:b], v_ref[a:b], 4e-2)):
            err = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
            assert err < tol, (a, b, err)
    move_gpu, move_ref = p_gpu - p0, p_ref - p0
    # every move is at most lr_t / (1 - b1^t) * |m_hat| / sqrt(v_hat) <= ~lr per step
    assert np.all(np.abs(move_gpu) <= 3.5 * lr)
    well = np.abs(g_bf) > 20.0 * np.abs(g_bf - g_64) + 1e-7
    assert well.mean() > 0.5, well.mean()
    bad = np.abs(move_gpu - move_ref) > 2e-2 * np.abs(move_ref) + 1e-9
    assert np.mean(bad[well]) < 0.01, np.mean(bad[well])
    # a plausible slip in the update (no bias correction, say) moves the first
    # step by ~3x, far outside this agreement
    assert np.median(np.abs(move_gpu[well] / move_ref[well] - 1.0)) < 1e-3
