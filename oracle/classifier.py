"""Learned bucket classifier: features, labels and a small MLP, in FP64.

Not in the paper.  The paper decides that a bucket holds a single mode by the
ratio-magnitude test of eq. (42).  The learned classifier replaces that test
with a network applied to the same ratios; the plain test stays the fallback.

Features of candidate bucket h (8 numbers).  With r_s = F_s[h] / F_0[h] and the
decoded unwrapped frequency y (eq. (41), refined by the K eps ladder when
present), the decoded phase is removed from a ratio of a set shifted by K eps
along axis n:  z = r exp(-i pi K y_n / N^d1)  (= 1 for a bucket with one mode).
The four ratios used are the coarse and fine shifts of the projection axis m
and of the axis n* != m whose fine ratio magnitude is furthest from 1 (ties by
the smaller n; n* = m when d2 = 1; "fine" is the coarse set without a ladder).
Each z gives asinh((Re z - 1) / s) and asinh(Im z / s), s the feature scale.

Label: 1 iff exactly one mode of the residual (planted modes minus the
registry, with |coefficient| >= eta) falls into bucket h.

Network: 8 -> 64 -> 64 -> 2 with ReLU; parameters in one flat vector
[W1 (64x8), b1 (64), W2 (64x64), b2 (64), W3 (2x64), b3 (2)], row-major.
The GPU stores them in BF16 and accumulates in FP32; this module evaluates
the same network in FP64 on BF16-rounded parameters and inputs.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_H, N_OUT = 8, 64, 2
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def bf16_round(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases (a starting point for training)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SIZES:
        if name.startswith("W"):
            parts.append(rng.normal(0.0, math.sqrt(2.0 / shape[1]), size=shape).ravel())
        else:
            parts.append(np.zeros(shape).ravel())
    return np.concatenate(parts)


def forward(theta, X):
    """Logits [n, 2] and the activations needed by `backward`."""
    P = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["W3"].T + P["b3"]
    return z, (X, a1, h1, a2, h2)


def prob_single(theta, X) -> np.ndarray:
    z, _ = forward(theta, X)
    return 1.0 / (1.0 + np.exp(z[:, 0] - z[:, 1]))


def loss_and_grad(theta, X, y):
    """Mean softmax cross-entropy over the batch and its gradient (flat)."""
    P = unpack(theta)
    z, (X, a1, h1, a2, h2) = forward(theta, X)
    n = X.shape[0]
    zmax = z.max(axis=1, keepdims=True)
    e = np.exp(z - zmax)
    sm = e / e.sum(axis=1, keepdims=True)
    y = np.asarray(y, dtype=np.int64)
    loss = float(np.mean(-np.log(sm[np.arange(n), y])))
    dz = sm.copy()
    dz[np.arange(n), y] -= 1.0
    dz /= n
    g = {}
    g["W3"] = dz.T @ h2
    g["b3"] = dz.sum(axis=0)
    dh2 = dz @ P["W3"] * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = dh2 @ P["W2"] * (a1 > 0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(axis=0)
    return loss, np.concatenate([g[name].ravel() for name, _ in SIZES])


def _arg(z: complex) -> float:
    th = math.atan2(z.imag, z.real)
    return -math.pi if th >= math.pi else th


def bucket_features(F, h: int, y, m: int, d2: int, ladder_K: int, NB: int,
                    scale: float) -> np.ndarray:
    """The 8 features of bucket h (F: spectra [S+1][p], y: decoded unwrapped frequency)."""
    F0 = complex(F[0][h])
    lad = ladder_K > 1

    def set_of(n, fine):
        return (d2 + n) if (fine and lad) else n

    def z(n, fine):
        K = ladder_K if (fine and lad) else 1
        r = complex(F[set_of(n, fine)][h]) / F0
        q = (K * int(y[n - 1])) % (2 * NB)
        return r * complex(math.cos(-math.pi * q / NB), math.sin(-math.pi * q / NB))

    others = [n for n in range(1, d2 + 1) if n != m] or [m]
    dev = [abs(abs(complex(F[set_of(n, True)][h]) / F0) - 1.0) for n in others]
    nstar = others[int(np.argmax(dev))]
    out = []
    for n, fine in ((m, False), (m, True), (nstar, False), (nstar, True)):
        zz = z(n, fine)
        out += [math.asinh((zz.real - 1.0) / scale), math.asinh(zz.imag / scale)]
    return np.array(out)


def bucket_label(h: int, p: int, m: int, y_planted, a_planted, R: dict, eta: float) -> int:
    """1 iff exactly one residual mode (planted minus R, |coeff| >= eta) lies in bucket h."""
    count = 0
    planted = {}
    for y, a in zip(y_planted, a_planted):
        key = tuple(int(v) for v in y)
        planted[key] = a
        res = a - R.get(key, 0.0)
        if abs(res) >= eta and key[m - 1] % p == h:
            count += 1
    for key, a in R.items():
        if key not in planted and abs(a) >= eta and key[m - 1] % p == h:
            count += 1
    return int(count == 1)
