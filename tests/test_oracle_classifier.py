"""Pins of the oracle's learned-classifier pieces (features, labels, FP64 MLP)."""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import classifier as C


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-6, 6, size=2000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16_round(x), ref)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = C.init_params(3) + rng.normal(scale=0.05, size=C.N_PARAMS)
    X = rng.normal(size=(32, 8))
    y = rng.integers(0, 2, size=32)
    loss, g = C.loss_and_grad(theta, X, y)
    idx = rng.choice(C.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (C.loss_and_grad(tp, X, y)[0] - C.loss_and_grad(tm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd)


def test_loss_closed_form():
    # zero weights and biases b3 = (u, v): softmax CE = log(1 + e^{v-u}) for label 0
    theta = np.zeros(C.N_PARAMS)
    theta[-2:] = [0.3, -1.1]
    loss, _ = C.loss_and_grad(theta, np.ones((4, 8)), np.zeros(4, dtype=int))
    assert abs(loss - math.log(1 + math.exp(-1.1 - 0.3))) < 1e-12


def _round_one(w, a, P):
    col = []
    oracle.multiphaseshift(w, a, P, collect=col, keep_spectra=True)
    return col


def test_features_vanish_on_noiseless_singletons():
    w, a = workloads.planted_signal(4001, 0, 6, 4096, 200, (1.0, 2.0))
    P = oracle.Params(d=6, N=4096, k=200, c=3.0, ladder_K=64, tau=1e-3, robust=True)
    col = _round_one(w, a, P)
    X = np.array([c[2] for c in col])
    lab = np.array([c[3] for c in col])
    assert lab.sum() > 0 and (lab == 0).sum() > 0
    # one mode: z = 1 exactly up to rounding -> features ~0 (scale 1e-3)
    assert np.abs(X[lab == 1]).max() < 1e-6
    # several modes: some feature is far from 0
    assert np.all(np.abs(X[lab == 0]).max(axis=1) > 1e-3)


def test_labels_count_residual_modes():
    w, a = workloads.planted_signal(4002, 0, 3, 256, 60, (1.0, 2.0))
    P = oracle.Params(d=3, N=256, k=60, c=2.0)
    col = []
    r = oracle.multiphaseshift(w, a, P, collect=col)
    y = oracle.unwrap(w, 1, 256)
    tr = {t["i"]: t for t in r.trace}
    # round 1: the registry is empty, so the label is "exactly one planted y_m = h mod p"
    for (i, h, x, lab, acc, _) in col:
        if i != 1:
            continue
        p, m = tr[1]["p"], tr[1]["m"]
        assert lab == int(np.sum(np.mod(y[:, m - 1], p) == h) == 1)


def test_plain_accepts_follow_labels_noiseless():
    # noiseless: the plain test accepts a bucket essentially iff it holds one mode
    w, a = workloads.planted_signal(4003, 0, 4, 1024, 256, (1.0, 2.0))
    col = []
    oracle.multiphaseshift(w, a, oracle.Params(d=4, N=1024, k=256, c=5.0), collect=col)
    lab = np.array([c[3] for c in col])
    acc = np.array([c[4] for c in col])
    assert np.mean(lab == acc) > 0.98
