"""Partial unwrapping, Section 4.1.2, eqs. (35), (36), (38).

The d coordinates are split into d2 = d / d1 consecutive blocks of d1.  Block
q (0-based) is unwrapped to the single coordinate

    y_q = sum_{r < d1} w_{d1 q + r} N^r            (eq. (35), 0-based indices)

which is injective on [-N/2, N/2)^d1 (balanced base-N digits).  In time, the
same map reads t_l = N^r t~_q for l = d1 q + r (eq. (36); the block index of
l is floor(l / d1) in 0-based terms).

Reading: eq. (35)/(38) use powers N^0 .. N^(d1-1); the sampling lines of the
MultiPhaseshift listing write N^1 .. N^d1, which would scale y by N and break
the bound |y| < 1/(2 eps).  The oracle follows eq. (35).
"""
from __future__ import annotations

import numpy as np


def unwrap_matrix(d: int, d1: int, N: int) -> np.ndarray:
    """U in Z^{d x d2} with U[d1 q + r, q] = N^r, so that y = U^T w."""
    if d % d1:
        raise ValueError("d must be a multiple of d1")
    d2 = d // d1
    U = np.zeros((d, d2), dtype=object)
    for q in range(d2):
        for r in range(d1):
            U[d1 * q + r, q] = int(N) ** r
    return U


def unwrap(w: np.ndarray, d1: int, N: int) -> np.ndarray:
    """y = U^T w for each row of w (int64 [k, d] -> int64 [k, d2]), eq. (35)."""
    w = np.asarray(w, dtype=np.int64)
    k, d = w.shape
    d2 = d // d1
    y = np.zeros((k, d2), dtype=np.int64)
    for q in range(d2):
        for r in range(d1):
            y[:, q] += w[:, d1 * q + r] * (int(N) ** r)
    return y


def wrap(y: np.ndarray, d1: int, N: int) -> np.ndarray:
    """Inverse of eq. (35): balanced base-N digits in [-N/2, N/2)."""
    y = np.asarray(y, dtype=np.int64)
    k, d2 = y.shape
    w = np.zeros((k, d2 * d1), dtype=np.int64)
    half = N // 2
    for q in range(d2):
        rest = y[:, q].copy()
        for r in range(d1):
            digit = np.mod(rest + half, N) - half
            w[:, d1 * q + r] = digit
            rest = (rest - digit) // N
        if np.any(rest != 0):
            raise ValueError("value outside the unwrapped range")
    return w


def y_range(N: int, d1: int) -> tuple[int, int]:
    """Inclusive range of an unwrapped coordinate: [-(N/2) S, (N/2 - 1) S], S = sum N^r."""
    S = sum(int(N) ** r for r in range(d1))
    return -(N // 2) * S, (N // 2 - 1) * S
