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
    return 0.5 * x * (1.0 + np.tanh(C0 * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    u = C0 * (x + 0.044715 * x ** 3)
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
