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
