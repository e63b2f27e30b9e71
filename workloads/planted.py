"""Random k-sparse d-dimensional trigonometric polynomials.

The signal model is the one of the paper's problem statement (Section 4.1.2,
eq. (32)): f(t) = sum_j a_j exp(2 pi i w_j . t) with integer frequency vectors
w_j in [-N/2, N/2)^d and complex coefficients a_j.  The empirical section
(Section 5) draws w_j uniformly and a_j = exp(2 pi i theta_j) with theta_j
uniform in [0, 1); the measured configurations widen |a_j| to a uniform range.

Frequencies inside one signal are distinct (drawn without replacement by
rejecting repeated rows).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class PlantedBatch:
    """A batch of B planted signals stored back to back.

    freqs:    int64 [total, d]     planted frequency vectors
    coeffs:   complex128 [total]   planted coefficients
    mode_off: int64 [B + 1]        signal b owns rows mode_off[b]:mode_off[b+1]
    k:        int32 [B]            sparsity handed to the method
    sigma:    float64 [B]          complex noise standard deviation per sample
    seed:     int                  key material of the per-sample noise stream
    d, N:     dimension and per-dimension bandwidth
    """

    freqs: np.ndarray
    coeffs: np.ndarray
    mode_off: np.ndarray
    k: np.ndarray
    sigma: np.ndarray
    seed: int
    d: int
    N: int

    @property
    def B(self) -> int:
        return int(self.k.shape[0])

    def signal(self, b: int):
        lo, hi = int(self.mode_off[b]), int(self.mode_off[b + 1])
        return self.freqs[lo:hi], self.coeffs[lo:hi]


def _distinct_rows(rng: np.random.Generator, k: int, d: int, N: int) -> np.ndarray:
    half = N // 2
    w = rng.integers(-half, half, size=(k, d), dtype=np.int64)
    # Reject repeated rows and redraw them until all k rows are distinct.
    for _ in range(1000):
        _, first = np.unique(w, axis=0, return_index=True)
        if first.size == k:
            return w
        dup = np.ones(k, dtype=bool)
        dup[first] = False
        w[dup] = rng.integers(-half, half, size=(int(dup.sum()), d), dtype=np.int64)
    raise RuntimeError("could not draw distinct frequencies; k too large for N^d")


def planted_signal(seed: int, index: int, d: int, N: int, k: int,
                   mag: tuple[float, float] = (1.0, 1.0)):
    """Draw one signal: (freqs int64[k, d], coeffs complex128[k]).

    The generator is keyed by (seed, index) so that signal `index` of a batch
    is the same whatever the batch size.
    """
    if N < 2 or N % 2:
        raise ValueError("N must be even and >= 2")
    if k < 0 or k > N ** min(d, 60):
        raise ValueError("bad sparsity")
    rng = np.random.default_rng([int(seed), int(index)])
    w = _distinct_rows(rng, k, d, N)
    lo, hi = mag
    r = rng.uniform(lo, hi, size=k) if hi > lo else np.full(k, float(lo))
    theta = rng.uniform(0.0, 1.0, size=k)
    a = r * np.exp(2j * np.pi * theta)
    return w, a.astype(np.complex128)


def planted_batch(seed: int, B: int, d: int, N: int, k, mag=(1.0, 1.0),
                  sigma=0.0) -> PlantedBatch:
    """Draw B signals.  `k` is an int or a length-B sequence; `sigma` likewise."""
    ks = np.broadcast_to(np.asarray(k, dtype=np.int64), (B,)).copy()
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (B,)).copy()
    fs, cs = [], []
    off = np.zeros(B + 1, dtype=np.int64)
    for b in range(B):
        w, a = planted_signal(seed, b, d, N, int(ks[b]), mag)
        fs.append(w)
        cs.append(a)
        off[b + 1] = off[b] + w.shape[0]
    freqs = np.concatenate(fs, axis=0) if fs else np.zeros((0, d), np.int64)
    coeffs = np.concatenate(cs) if cs else np.zeros(0, np.complex128)
    return PlantedBatch(freqs=np.ascontiguousarray(freqs), coeffs=coeffs, mode_off=off,
                        k=ks.astype(np.int32), sigma=sig, seed=int(seed), d=d, N=N)


def uneven_k(seed: int, B: int, lo: int, hi: int) -> np.ndarray:
    """Per-signal sparsities drawn uniformly from the integers lo..hi."""
    rng = np.random.default_rng([int(seed), 0x6B])
    return rng.integers(lo, hi + 1, size=B).astype(np.int32)


def uniform_sigma(seed: int, B: int, lo: float, hi: float) -> np.ndarray:
    rng = np.random.default_rng([int(seed), 0x5D])
    return rng.uniform(lo, hi, size=B)


def rectangle_batch(seed: int, B: int, N: int, r: int, mag=(1.0, 2.0),
                    sigma=0.0) -> PlantedBatch:
    """B two-dimensional signals whose k = r^2 frequencies are the grid X x Y of r
    distinct first and r distinct second coordinates (Section 3.3's worst case:
    every frequency is a vertex of axis-aligned rectangles, so each one shares its
    projection onto either axis with r - 1 others)."""
    if r < 1 or r > N:
        raise ValueError("bad grid size")
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (B,)).copy()
    fs, cs = [], []
    off = np.zeros(B + 1, dtype=np.int64)
    half = N // 2
    for b in range(B):
        rng = np.random.default_rng([int(seed), int(b), 0x7E])
        xs = rng.choice(np.arange(-half, half), size=r, replace=False)
        ys = rng.choice(np.arange(-half, half), size=r, replace=False)
        w = np.stack(np.meshgrid(xs, ys, indexing="ij"), axis=-1).reshape(-1, 2).astype(np.int64)
        lo, hi = mag
        rad = rng.uniform(lo, hi, size=r * r) if hi > lo else np.full(r * r, float(lo))
        a = rad * np.exp(2j * np.pi * rng.uniform(0.0, 1.0, size=r * r))
        fs.append(w)
        cs.append(a.astype(np.complex128))
        off[b + 1] = off[b] + r * r
    return PlantedBatch(freqs=np.ascontiguousarray(np.concatenate(fs)),
                        coeffs=np.concatenate(cs), mode_off=off,
                        k=np.full(B, r * r, np.int32), sigma=sig, seed=int(seed), d=2, N=N)
