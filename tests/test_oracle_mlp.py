"""Pins of the FP64 surrogate reference (oracle/mlp.py): its backward pass
against central finite differences of its forward pass, its activation
derivative against finite differences, and the BF16 rounding helper against
exact bit arithmetic."""
import numpy as np

from oracle import mlp as M


def _random_params(rng, scale=0.5):
    return rng.normal(0.0, scale, M.N_PARAMS) / np.sqrt(np.repeat(
        [96, 1, 64, 1, 64, 1, 64, 1], [6144, 64, 4096, 64, 4096, 64, 64, 1]))


def test_gelu_grad_matches_finite_differences():
    x = np.linspace(-6, 6, 1001)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(x))) < 1e-8
    # limits: gelu(x) -> x for large x, -> 0 for very negative x
    assert abs(M.gelu(np.array([10.0]))[0] - 10.0) < 1e-12
    assert abs(M.gelu(np.array([-10.0]))[0]) < 1e-12


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = _random_params(rng)
    X = rng.normal(0, 0.5, (37, 96))
    t = rng.normal(0, 1, 37)
    loss, g = M.loss_and_grad(p, X, t)
    idx = np.concatenate([rng.choice(6144, 20, replace=False),             # W1
                          6144 + rng.choice(64, 5, replace=False),         # b1
                          6208 + rng.choice(4096, 15, replace=False),      # W2
                          10304 + rng.choice(64, 5, replace=False),        # b2
                          10368 + rng.choice(4096, 15, replace=False),     # W3
                          14464 + rng.choice(64, 5, replace=False),        # b3
                          14528 + rng.choice(64, 5, replace=False), [14592]])  # w4, b4
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (M.loss_and_grad(pp, X, t)[0] - M.loss_and_grad(pm, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-9, 1.0 + 3 * 2**-9, -3.14159, 0.0], np.float64)
    r = M.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0 + 2**-7 or r[1] == 1.0  # 1 + 2^-8 is a tie: rounds to even (1.0)
    assert r[1] == 1.0
    assert r[2] == 1.0                        # below half an ulp
    assert r[3] == 1.0 + 2**-7                # above half an ulp
    assert abs(r[4] + 3.140625) < 1e-12
    assert r[5] == 0.0


def test_first_order_expansion_error_is_second_order(oracle_mod):
    """The first-order coupling C' of eq. (drifta) approaches the product-form
    coupling of eq. (LIBOR-drift-PT) with an error of order ell^2: its relative
    error halves when all forwards halve (Section 3.2)."""
    import workloads
    rel = []
    for f in (4e-3, 2e-3, 1e-3):
        ts = workloads.learned_drift()
        ts.L0 = ts.L0 * f
        o = oracle_mod.Oracle(ts)
        for k in (0, 137):
            m = k // ts.steps_per_period
            L = np.asarray(ts.L0, dtype=np.float64)
            C = -o.drift(k, L) - o.kappa[k]
            ell = ts.delta * L / (1 + ts.delta * L)
            ell[:m] = 0.0
            C1 = M.first_order_coupling(ell[None, :], np.asarray(ts.vol[k]), ts)[0]
            i = m  # first live rate: the longest coupling sum
            assert np.sign(C1[i]) == np.sign(C[i])
            rel.append(abs(C1[i] / C[i] - 1.0))
            assert C[-1] == 0.0 and C1[-1] == 0.0
    r = np.array(rel).reshape(3, 2)
    ratios = r[:-1] / r[1:]
    assert np.all(np.abs(ratios - 2.0) < 0.05), ratios
    assert np.all(r[0] < 1e-3)


def test_surrogate_paths_with_empty_box_are_full_euler(oracle_mod):
    """With an empty trust box every coupling falls back to the quadrature, so
    the surrogate scheme must reproduce the FULL Euler paths of the C oracle
    (same streams, same payoff sums) up to FP64 rounding order."""
    import workloads
    ts = workloads.learned_drift()
    o = oracle_mod.Oracle(ts)
    rng = np.random.default_rng(5)
    p = _random_params(rng)
    lo, hi = np.ones(40), -np.ones(40)
    sums, Lf, Df = M.surrogate_paths(o, p, lo, hi, 0.01, np.arange(8))
    ref = o.price_sums(0, 8)
    Lo, Do = o.paths(0, np.arange(8))
    assert np.allclose(Lf, Lo, rtol=1e-12, atol=0)
    assert np.allclose(Df, Do, rtol=1e-12, atol=0)
    assert np.allclose(sums["sum_p"], ref["sum_p"], rtol=1e-10, atol=1e-300)
    assert np.array_equal(sums["n_itm"], ref["n_itm"])
    assert np.allclose(sums["sum_mart"], ref["sum_mart"], rtol=1e-12)
    assert sums["fallbacks"] == 8 * sum(39 - k // 10 for k in range(400) if k // 10 < 39)
    # sparse path indices take the same streams as a contiguous range
    s2, L2, _ = M.surrogate_paths(o, p, lo, hi, 0.01, np.array([3, 6]))
    assert np.allclose(L2, Lo[[3, 6]], rtol=1e-12, atol=0)


def test_surrogate_paths_first_order_close_to_full(oracle_mod):
    """With the first-order coupling alone the fixings stay within the O(ell^2)
    drift error of the FULL paths; with a network that outputs exactly zero
    (all weights 0) the surrogate scheme is the first-order scheme."""
    import workloads
    ts = workloads.learned_drift()
    o = oracle_mod.Oracle(ts)
    big = np.full(40, 1e30)
    s1, L1, _ = M.surrogate_paths(o, np.zeros(M.N_PARAMS), -big, big, 1.0, np.arange(4))
    s0, L0f, _ = M.surrogate_paths(o, None, -big, big, 1.0, np.arange(4), use_net=False)
    assert np.array_equal(L1, L0f)
    Lo, _ = o.paths(0, np.arange(4))
    d = np.abs(L0f / Lo - 1.0)
    assert 0 < d.max() < 1e-3


def test_adam_step_and_cosine_schedule_match_torch():
    """The oracle's Adam step and cosine learning-rate decay against
    torch.optim.Adam with CosineAnnealingLR (eta_min = lr / 100), FP64, on a
    sequence of gradients with a wide spread of magnitudes."""
    import torch
    rng = np.random.default_rng(4)
    n, steps, lr = 300, 25, 2e-3
    p0 = rng.normal(0, 1, n)
    grads = [rng.normal(0, 1, n) * 10.0 ** rng.uniform(-9, 1, n) for _ in range(steps)]
    w = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=steps, eta_min=lr / 100)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    # torch forms the averages by lerp, m + (1 - b1)(g - m): the same value up
    # to rounding relative to the magnitudes summed so far
    g_abs, g_sq = np.zeros(n), np.zeros(n)
    for t in range(steps):
        g_abs += np.abs(grads[t])
        g_sq += grads[t] ** 2
        assert abs(M.cosine_lr(lr, t, steps) - opt.param_groups[0]["lr"]) <= 1e-15
        w.grad = torch.tensor(grads[t], dtype=torch.float64)
        opt.step()
        sched.step()
        p, m, v = M.adam_step(p, m, v, grads[t], t + 1, M.cosine_lr(lr, t, steps))
        st = opt.state[w]
        assert np.all(np.abs(st["exp_avg"].numpy() - m) <= 1e-14 * g_abs)
        assert np.all(np.abs(st["exp_avg_sq"].numpy() - v) <= 1e-14 * g_sq)
        assert np.all(np.abs(w.detach().numpy() - p) <= 1e-13 * (np.abs(p) + lr * (t + 1)))
    # a plausible slip (no bias correction) is far outside that agreement
    p1, _, _ = M.adam_step(p0, np.zeros(n), np.zeros(n), grads[0], 1, lr)
    m_raw = 0.1 * grads[0]
    p_nobc = p0 - lr * m_raw / (np.sqrt(0.001 * grads[0] ** 2) + 1e-8)
    assert np.max(np.abs(p1 - p_nobc)) > lr


def test_minibatch_draws_are_uniform_and_reproducible(oracle_mod):
    """Minibatch indices from the oracle's Philox: in range, the same for the
    same (seed, step), different across steps, and uniform (chi-square over 16
    cells of 4096 draws)."""
    a = M.minibatch(oracle_mod.philox4x32_10, 7, 3, 4096, 1000003)
    assert np.array_equal(a, M.minibatch(oracle_mod.philox4x32_10, 7, 3, 4096, 1000003))
    assert a.min() >= 0 and a.max() < 1000003
    b = M.minibatch(oracle_mod.philox4x32_10, 7, 4, 4096, 1000003)
    assert np.mean(a == b) < 0.01
    counts = np.bincount(a * 16 // 1000003, minlength=16)
    chi2 = np.sum((counts - 256.0) ** 2 / 256.0)
    assert chi2 < 45.0          # 15 degrees of freedom: p ~ 1e-4


def test_training_loop_reduces_loss_and_follows_the_gradient(oracle_mod):
    """The oracle's training loop on a small regression: the loss falls, and
    its first move is -lr g / (|g| + eps), i.e. -lr sign(g) wherever the
    gradient is not tiny (after bias correction the first moments are g and g^2)."""
    rng = np.random.default_rng(5)
    p0 = _random_params(rng, 0.3)
    feat = M.bf16(rng.normal(0, 0.5, (512, 96)))
    labels = 3.0 * np.tanh(feat[:, 1] - feat[:, 2]) + 0.1
    p1, m1, v1, l1 = M.train(p0, feat, labels, 2.0, 1, 128, 1e-3, 9, oracle_mod.philox4x32_10)
    idx = M.minibatch(oracle_mod.philox4x32_10, 9, 1, 128, 512)
    _, g = M.loss_and_grad(p0, feat[idx], labels[idx] / 2.0, bf=True)
    assert np.allclose(p1 - p0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-18)
    big = np.abs(g) > 1e-4
    assert np.allclose((p1 - p0)[big], -1e-3 * np.sign(g[big]), rtol=1e-4, atol=0)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    _, _, _, losses = M.train(p0, feat, labels, 2.0, 60, 128, 3e-3, 9, oracle_mod.philox4x32_10)
    assert losses[-10:].mean() < 0.5 * losses[:5].mean()
