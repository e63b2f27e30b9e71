"""Black-box access to the planted signal, evaluated directly in FP64.

f(t) = sum_j a_j exp(2 pi i w_j . t) for t in R^d (eq. (32)).  The oracle
forms the real sample points t of the MultiPhaseshift sampling lines and
evaluates the exponential sum at them; it does no integer argument reduction
(the HIP sampler does, so the two take different routes to the same values).
"""
from __future__ import annotations

import numpy as np

from .unwrapping import unwrap_matrix


def evaluate(freqs: np.ndarray, coeffs: np.ndarray, t: np.ndarray,
             chunk: int = 2048) -> np.ndarray:
    """f at the rows of t (float64 [n, d]) -> complex128 [n]."""
    freqs = np.asarray(freqs, dtype=np.float64)
    coeffs = np.asarray(coeffs, dtype=np.complex128)
    t = np.asarray(t, dtype=np.float64)
    out = np.empty(t.shape[0], dtype=np.complex128)
    for lo in range(0, t.shape[0], chunk):
        ph = t[lo:lo + chunk] @ freqs.T
        out[lo:lo + chunk] = np.exp(2j * np.pi * ph) @ coeffs
    return out


def sample_points(d: int, d1: int, N: int, p: int, m: int, shift_axis: int,
                  shift: float, blocks=None, order=None, tilt=None) -> np.ndarray:
    """Points of one sampling line, float64 [p, d].

    t_h = (h/p) U e_m + shift U e_n  for h = 0..p-1 (eq. (41) with the partial
    unwrapping of eq. (36)); m and n = shift_axis are 1-based unwrapped axes,
    shift = 0 gives the unshifted line.  0-based h with h/p is the reading of
    eq. (2); the listings' (h-1)/p for h = 1..p is the same set of points.
    blocks / order: a general partition; tilt: the rotation of Section 3.3 (see
    unwrap_matrix).
    """
    U = unwrap_matrix(d, d1, N, blocks, order, tilt).astype(np.float64)
    h = np.arange(p, dtype=np.float64)[:, None]
    t = (h / p) * U[:, m - 1][None, :]
    if shift != 0.0:
        t = t + shift * U[:, shift_axis - 1][None, :]
    return t
