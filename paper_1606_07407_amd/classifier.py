"""Training data and training of the learned bucket classifier, on the GPU.

Bucket features come from the method itself: sfft_export_bucket_features runs
the recovery with the plain ratio test on synthetic signals (d = 6, N = 4096,
k = 2000, |a| ~ U[1, 2], noise sigma ~ U[0, 1e-2] per signal), and every
candidate bucket of every round becomes one (features, label) row.
Training runs the project's forward/backward and Adam kernels
(sfft_mlp_train).  Only device memory and the stream come from PyTorch.
"""
from __future__ import annotations

import numpy as np

from . import sfft

# parameters of the feature-generating recovery (bucket test, shifts, primes)
TRAIN_RECIPE = dict(d=6, N=4096, k=2000, mag=(1.0, 2.0), sigma=(0.0, 1e-2), c=2.0,
                    ladder_K=64, tau=1e-3, eta=1e-3, p_min=101, robust=1)


def export_features(n_rows: int, seed: int = 4000, batch: int = 256, recipe=None,
                    device="cuda"):
    """At least n_rows (features, labels) rows as device tensors, plus per-row signal ids."""
    import torch

    import workloads
    r = dict(TRAIN_RECIPE if recipe is None else recipe)
    params = sfft.Params(d=r["d"], N=r["N"], k_max=r["k"], c=r["c"], p_min=r["p_min"],
                         ladder_K=r["ladder_K"], tau=r["tau"], eta=r["eta"],
                         precision=sfft.SFFT_FP32, robust=r["robust"])
    plan = sfft.sfft_plan_create(params, max_batch=batch)
    feats, labels, sig = [], [], []
    total, b0 = 0, 0
    while total < n_rows:
        s = seed + b0
        sg = workloads.planted.uniform_sigma(s, batch, *r["sigma"])
        pb = workloads.planted_batch(s, batch, r["d"], r["N"], r["k"], r["mag"], sg)
        cap = batch * 4 * r["k"]
        out = sfft.sfft_export_bucket_features(plan, sfft.DeviceBatch.from_planted(pb, device),
                                               cap)
        n = int(out["feat_count"].item())
        n = min(n, cap)
        feats.append(out["feat"][:n].clone())
        labels.append(out["label"][:n].clone())
        sig.append(out["feat_meta"][:n, 0].to(torch.int64) + b0)
        total += n
        b0 += batch
    plan.close()
    return torch.cat(feats), torch.cat(labels), torch.cat(sig)


def init_weights(seed: int = 0, device="cuda"):
    """He-normal weights and zero biases, as a BF16 device tensor."""
    import torch
    rng = np.random.default_rng(seed)
    parts = []
    for n_out, n_in in ((64, 8), (64, 64), (2, 64)):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / n_in), size=n_out * n_in))
        parts.append(np.zeros(n_out))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == sfft.SFFT_MLP_PARAMS
    return torch.tensor(theta, device=device).to(torch.bfloat16)


def train(x, y, epochs: int = 8, batch: int = 4096, lr: float = 2e-3, seed: int = 1,
          init_seed: int = 0):
    """Train a fresh network on (x, y); returns (BF16 weights, per-epoch mean losses)."""
    w = init_weights(init_seed, device=x.device)
    hist = sfft.sfft_mlp_train(w, x, y, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return w, hist.cpu().numpy()


def accuracy(w, x, y, threshold: float = 0.5) -> float:
    p = sfft.sfft_mlp_forward(w, x)
    return float(((p > threshold) == (y == 1)).float().mean().item())
