"""FP64 reference of the drift surrogate network (forward and backward).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).  Plain numpy matrix
products as library steps.  Architecture: 96 inputs -> 64 -> 64 -> 64 -> 1,
tanh-form GELU  gelu(x) = x/2 (1 + tanh(sqrt(2/pi)(x + 0.044715 x^3))),
loss = sum (y - t)^2 / (2 n).  Parameter vector (FP32 on the device):
W1[64][96] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] w4[64] b4.

``bf16=True`` reproduces the device's operand rounding: the weights of the
three hidden layers, the inputs, the hidden activations and the backward
pre-activation gradients are rounded to bfloat16 (round to nearest even)
where the device feeds them to its BF16 matrix cores; products are then
accumulated exactly here (FP64) rather than in FP32.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_HID = 96, 64
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("w4", (N_HID,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x):
    """Round to bfloat16 (nearest even) and back to float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


C0 = math.sqrt(2.0 / math.pi)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(C0 * (x + 0.044715 * x * x * x)))


def gelu_grad(x):
    u = C0 * (x + 0.044715 * x * x * x)
    t = np.tanh(u)
    du = C0 * (1.0 + 3.0 * 0.044715 * x * x)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du


def forward(p, X, bf=False):
    """Outputs y[n] and the intermediates needed by backward."""
    w = unpack(p)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    X = r(X)
    z1 = X @ r(w["W1"]).T + w["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ r(w["W2"]).T + w["b2"]
    h2 = r(gelu(z2))
    z3 = h2 @ r(w["W3"]).T + w["b3"]
    h3 = r(gelu(z3))
    y = h3 @ w["w4"] + w["b4"][0]
    return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3)


def loss_and_grad(p, X, t, bf=False):
    """Loss sum (y - t)^2 / (2 n) and its gradient with respect to p."""
    w = unpack(p)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    y, c = forward(p, X, bf)
    n = len(t)
    d = y - np.asarray(t, dtype=np.float64)
    loss = float(np.sum(d * d) / (2 * n))
    dy = d / n
    g = {"w4": c["h3"].T @ dy, "b4": np.array([dy.sum()])}
    dz3 = np.outer(dy, w["w4"]) * gelu_grad(c["z3"])
    g["W3"] = r(dz3).T @ c["h2"]
    g["b3"] = dz3.sum(axis=0)
    dz2 = (r(dz3) @ r(w["W3"])) * gelu_grad(c["z2"])
    g["W2"] = r(dz2).T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (r(dz2) @ r(w["W2"])) * gelu_grad(c["z1"])
    g["W1"] = r(dz1).T @ c["X"]
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


# ---------------------------------------------------------------------------
# Euler paths with the surrogate drift
# ---------------------------------------------------------------------------

def nig_kappa(u, alpha, beta, delta):
    """NIG cumulant kappa(u) = log E[e^{u H_1}] with the martingale location
    mu = -delta beta / gamma (Section 2's log moment generating function)."""
    gamma = math.sqrt(alpha * alpha - beta * beta)
    mu = -delta * beta / gamma
    u = np.asarray(u, dtype=np.float64)
    return mu * u + delta * (gamma - np.sqrt(alpha * alpha - (beta + u) ** 2))


def first_order_coupling(ell, lam, ts):
    """First-order expansion of the coupling (Section 3.2, eq. (drifta)):
    C'_i = sum_{l>i} ell_l [kappa(lam_i + lam_l) - kappa(lam_i) - kappa(lam_l)].
    ell: [..., N]; lam: [N]; returns [..., N]."""
    k1 = nig_kappa(lam, ts.alpha, ts.beta, ts.delta_nig)
    k2 = nig_kappa(lam[:, None] + lam[None, :], ts.alpha, ts.beta, ts.delta_nig)
    K2 = np.triu(k2 - k1[:, None] - k1[None, :], 1)     # [i, l], l > i only
    return ell @ K2.T


def features(tn, X, i):
    """Inputs of the network for rate i at normalised time tn and states X[n, 40]
    (log L_l - log L_l(0)); rates l <= i are zeroed; one-hot of i."""
    n = X.shape[0]
    f = np.zeros((n, N_IN))
    f[:, 0] = tn
    f[:, 2 + i:41] = X[:, i + 1:40]
    f[:, 41 + i] = 1.0
    return f


def surrogate_paths(o, params, lo, hi, sigma, paths, use_net=True):
    """FP64 Euler paths (eq. (LIBOR-drift-PT)) of the given path indices with
    the coupling C_i replaced by C'_i + sigma * net(features_i), or by C'_i alone
    when use_net is False; the last rate has no coupling.  A rate whose later
    rates leave the box [lo, hi] (compared in FP32, as the device compares)
    takes the quadrature coupling of the oracle instead.  The increments are the
    oracle's (same Philox streams).  Returns payoff sums in the layout of
    Oracle.price_sums and the per-path fixings (L_c, D_c), each [n, N].
    Needs a structure of 40 rates."""
    ts = o.ts
    N, s, K = o.N, o.s, o.K
    assert N == 40
    paths = np.asarray(paths, dtype=np.int64)
    n = len(paths)
    contiguous = n > 0 and np.array_equal(paths, paths[0] + np.arange(n))
    L0 = np.asarray(ts.L0, dtype=np.float64)
    delta = np.asarray(ts.delta, dtype=np.float64)
    strikes = np.asarray(ts.strikes, dtype=np.float64)
    lo32 = np.asarray(lo, dtype=np.float32)
    hi32 = np.asarray(hi, dtype=np.float32)
    T = np.concatenate([[0.0], np.asarray(ts.tenor, dtype=np.float64)])
    X = np.zeros((n, N))
    Lfix = np.zeros((n, N))
    Dfix = np.zeros((n, N))
    S = strikes.shape[1]
    sp = np.zeros((N, S)); sp2 = np.zeros((N, S)); itm = np.zeros((N, S))
    mart = np.zeros(N); mart2 = np.zeros(N)
    fallbacks = 0
    for k in range(K):
        m = k // s
        if contiguous:
            _, dH = o.increments(k, int(paths[0]), n)
        else:
            dH = np.array([o.increments(k, int(p), 1)[1][0] for p in paths])
        lam = np.asarray(ts.vol[k], dtype=np.float64)
        L = L0 * np.exp(X)
        ell = delta * L / (1.0 + delta * L)
        ell[:, :m] = 0.0
        C = first_order_coupling(ell, lam, ts)
        if use_net:
            tk = T[m] + (k - m * s) * (T[m + 1] - T[m]) / s
            tn = float(np.float32(tk / T[N]))
            rates = range(m, N - 1)
            if len(rates):
                y, _ = forward(params, np.concatenate([features(tn, X, i) for i in rates]), bf=True)
                C[:, m:N - 1] += sigma * y.reshape(len(rates), n).T
            X32 = X.astype(np.float32)
            out = ((X32 < lo32) | (X32 > hi32)).astype(np.int64)
            out[:, :m] = 0
            later = np.cumsum(out[:, ::-1], axis=1)[:, ::-1]     # later[p, i] = #out l >= i
            fb = np.zeros((n, N), dtype=bool)
            fb[:, :N - 1] = later[:, 1:] > 0
            fb[:, :m] = False
            for p in np.nonzero(fb.any(axis=1))[0]:
                b = o.drift(k, L[p])
                quad = -b - o.kappa[k]
                C[p, fb[p]] = quad[fb[p]]
            fallbacks += int(fb.sum())
        C[:, N - 1] = 0.0
        X[:, m:] += (-o.kappa[k, m:] - C[:, m:]) * o.dt[k] + lam[m:] * dH[:, None]
        if (k + 1) % s == 0:
            c = m
            Lc = L0[c] * np.exp(X[:, c])
            D = np.prod(1.0 + delta[c + 1:] * L0[c + 1:] * np.exp(X[:, c + 1:]), axis=1)
            Lfix[:, c], Dfix[:, c] = Lc, D
            pay = D[:, None] * np.maximum(Lc[:, None] - strikes[c][None, :], 0.0)
            sp[c] = pay.sum(axis=0)
            sp2[c] = (pay * pay).sum(axis=0)
            itm[c] = (Lc[:, None] > strikes[c][None, :]).sum(axis=0)
            mt = D * (1.0 + delta[c] * Lc)
            mart[c] = mt.sum()
            mart2[c] = (mt * mt).sum()
    sums = {"sum_p": sp, "sum_p2": sp2, "n_itm": itm, "sum_mart": mart, "sum_mart2": mart2,
            "n_paths": n, "fallbacks": fallbacks}
    return sums, Lfix, Dfix


# ---------------------------------------------------------------------------
# Training update (the surrogate's own optimiser; not part of the paper)
# ---------------------------------------------------------------------------

ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_step(p, m, v, g, t, lr, b1=ADAM_B1, b2=ADAM_B2, eps=ADAM_EPS):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) at step t = 1, 2, ...:
    exponential moving averages m, v of the gradient and of its square, their
    bias corrections m / (1 - b1^t) and v / (1 - b2^t), and the parameter move
    -lr m_hat / (sqrt(v_hat) + eps).  FP64; returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def cosine_lr(lr, t, n_steps, floor=0.01):
    """Learning rate of step t = 0 .. n_steps - 1 of a call: cosine decay from
    lr towards floor * lr, lr (floor + (1 - floor) (1 + cos(pi t / n_steps)) / 2)."""
    return lr * (floor + (1.0 - floor) * 0.5 * (1.0 + math.cos(math.pi * t / n_steps)))


def minibatch(philox, seed, step, batch, n_pairs):
    """Indices of the minibatch of Adam step `step` (1-based, counted over the
    network's life): draw j takes the Philox-4x32-10 words of counter
    (step, j, 1, 2 << 24) (tag 2 of the counter layout) under key (seed mod 2^32,
    seed div 2^32) and returns (w0 2^32 + w1) mod n_pairs -- a draw with
    replacement.  `philox(ctr, key)` is the oracle's generator."""
    key = (seed & 0xFFFFFFFF, seed >> 32)
    out = np.empty(batch, dtype=np.int64)
    for j in range(batch):
        w = philox((step & 0xFFFFFFFF, j, 1, 2 << 24), key)
        out[j] = ((int(w[0]) << 32) | int(w[1])) % n_pairs
    return out


def train(p, feat, labels, sigma, n_steps, batch, lr, seed, philox, step0=0, m=None, v=None):
    """The surrogate's training loop in FP64: per step t the minibatch of step
    step0 + t + 1, the loss sum (y - label / sigma)^2 / (2 batch) and its
    gradient through the network with the device's BF16 operand rounding
    (``loss_and_grad(..., bf=True)``), and an Adam step at the cosine-decayed
    learning rate.  Returns (p, m, v, losses)."""
    p = np.asarray(p, dtype=np.float64).copy()
    m = np.zeros_like(p) if m is None else np.asarray(m, dtype=np.float64).copy()
    v = np.zeros_like(p) if v is None else np.asarray(v, dtype=np.float64).copy()
    feat = np.asarray(feat, dtype=np.float64)
    labels = np.asarray(labels, dtype=np.float64)
    losses = []
    for t in range(n_steps):
        step = step0 + t + 1
        idx = minibatch(philox, seed, step, batch, len(labels))
        loss, g = loss_and_grad(p, feat[idx], labels[idx] / sigma, bf=True)
        p, m, v = adam_step(p, m, v, g, step, cosine_lr(lr, t, n_steps))
        losses.append(loss)
    return p, m, v, np.array(losses)
