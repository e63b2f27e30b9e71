"""Partial unwrapping, Section 4.1.2, eqs. (35), (36), (38).

The d coordinates are split into d2 = d / d1 consecutive blocks of d1.  Block
q (0-based) is unwrapped to the single coordinate

    y_q = sum_{r < d1} w_{d1 q + r} N^r            (eq. (35), 0-based indices)

which is injective on [-N/2, N/2)^d1 (balanced base-N digits).  In time, the
same map reads t_l = N^r t~_q for l = d1 q + r (eq. (36); the block index of
l is floor(l / d1) in 0-based terms).

General partitions (Section 4.1: the coordinates of a block need not be in
their natural order, and blocks need not have one size; Section 4.1.2, last
paragraph: d prime, components of different bandwidths): blocks of sizes
d_0, ..., d_{d2-1} (sum d) taken over a coordinate order pi (a permutation of
0..d-1).  Block q starts at s_q = d_0 + ... + d_{q-1} and

    y_q = sum_{r < d_q} w_{pi(s_q + r)} N^r,

of bandwidth N^{d_q}.  blocks=None is the uniform partition into blocks of d1,
order=None the natural order; together they are eq. (35).

Reading: eq. (35)/(38) use powers N^0 .. N^(d1-1); the sampling lines of the
MultiPhaseshift listing write N^1 .. N^d1, which would scale y by N and break
the bound |y| < 1/(2 eps).  The oracle follows eq. (35).
"""
from __future__ import annotations

import math

import numpy as np


def partition(d: int, d1: int, blocks=None, order=None):
    """(block sizes, coordinate order, block starts) of a partition of d coordinates."""
    if blocks is None:
        if d1 < 1 or d % d1:
            raise ValueError("d must be a multiple of d1")
        blocks = (int(d1),) * (d // d1)
    blocks = tuple(int(b) for b in blocks)
    if not blocks or any(b < 1 for b in blocks) or sum(blocks) != d:
        raise ValueError("block sizes must be positive and sum to d")
    order = tuple(range(d)) if order is None else tuple(int(x) for x in order)
    if sorted(order) != list(range(d)):
        raise ValueError("order must be a permutation of 0..d-1")
    starts = [0]
    for b in blocks:
        starts.append(starts[-1] + b)
    return blocks, order, tuple(starts)


def unwrap_matrix(d: int, d1: int, N: int, blocks=None, order=None,
                  tilt=None) -> np.ndarray:
    """U in Z^{d x d2} with U[pi(s_q + r), q] = N^r, so that y = U^T w; with
    tilt = (a, b, c) (d = 2) the scaled rotation of eq. (27)."""
    if tilt is not None:
        return tilt_matrix(tilt[0], tilt[1])
    blocks, order, starts = partition(d, d1, blocks, order)
    U = np.zeros((d, len(blocks)), dtype=object)
    for q, dq in enumerate(blocks):
        for r in range(dq):
            U[order[starts[q] + r], q] = int(N) ** r
    return U


def unwrap(w: np.ndarray, d1: int, N: int, blocks=None, order=None) -> np.ndarray:
    """y = U^T w for each row of w (int64 [k, d] -> int64 [k, d2]), eq. (35)."""
    w = np.asarray(w, dtype=np.int64)
    k, d = w.shape
    blocks, order, starts = partition(d, d1, blocks, order)
    y = np.zeros((k, len(blocks)), dtype=np.int64)
    for q, dq in enumerate(blocks):
        for r in range(dq):
            y[:, q] += w[:, order[starts[q] + r]] * (int(N) ** r)
    return y


def wrap(y: np.ndarray, d1: int, N: int, blocks=None, order=None) -> np.ndarray:
    """Inverse of eq. (35): balanced base-N digits in [-N/2, N/2)."""
    y = np.asarray(y, dtype=np.int64)
    k, d2 = y.shape
    d = d2 * d1 if blocks is None else sum(int(b) for b in blocks)
    blocks, order, starts = partition(d, d1, blocks, order)
    if len(blocks) != d2:
        raise ValueError("y has the wrong number of unwrapped coordinates")
    w = np.zeros((k, d), dtype=np.int64)
    half = N // 2
    for q, dq in enumerate(blocks):
        rest = y[:, q].copy()
        for r in range(dq):
            digit = np.mod(rest + half, N) - half
            w[:, order[starts[q] + r]] = digit
            rest = (rest - digit) // N
        if np.any(rest != 0):
            raise ValueError("value outside the unwrapped range")
    return w


def y_range(N: int, d1: int) -> tuple[int, int]:
    """Inclusive range of a coordinate unwrapped from a block of d1:
    [-(N/2) S, (N/2 - 1) S], S = sum N^r."""
    S = sum(int(N) ** r for r in range(d1))
    return -(N // 2) * S, (N // 2 - 1) * S


# ---- 2D tilting (Section 3.3, eqs. (21), (25), (27), Theorem 1) -------------------------
#
# The frequency plane is rotated by theta with sin theta = a/c, cos theta = b/c, (a, b, c)
# a Pythagorean triple, and scaled by c so that the rotated frequencies stay integers:
# the sampling lines run in coordinates t = U t~ with U = [[b, a], [-a, b]] (eq. (27)),
# so that y = U^T w = (b w_1 - a w_2, a w_1 + b w_2).  U U^T = c^2 I, hence
# w = U y / c^2 exactly (the listing's rotation back).  By Theorem 1, with b > 2N and
# gcd(a, b) = 1, no two frequencies of [-N/2, N/2)^2 share either rotated coordinate.


def pythagorean_tilt(N: int) -> tuple[int, int, int]:
    """The triple (a, b, c) with a^2 + b^2 = c^2, c > b > a >= 1, gcd(a, b) = 1 and
    b > 2N (Theorem 1) whose bandwidth a + b is smallest (ties: smaller b).

    Primitive triples are (m^2 - n^2, 2 m n, m^2 + n^2) with m > n >= 1 coprime and of
    opposite parity (Euclid); a + b >= m^2 > 8N beyond m = sqrt(8N) + 1, while the
    triple of n = ceil(sqrt(N)), m = n + 1 already has a + b <= 8N, so the search stops
    there."""
    best = None
    m_max = int(math.isqrt(8 * int(N))) + 2
    for m in range(2, m_max + 1):
        for n in range(1, m):
            if (m - n) % 2 == 0 or math.gcd(m, n) != 1:
                continue
            u, v, c = m * m - n * n, 2 * m * n, m * m + n * n
            for a, b in ((u, v), (v, u)):
                if b > 2 * N and a < b:
                    key = (a + b, b)
                    if best is None or key < best[0]:
                        best = (key, (a, b, c))
    return best[1]


def tilt_matrix(a: int, b: int) -> np.ndarray:
    """U of eq. (27) (scaled rotation), t = U t~: U = [[b, a], [-a, b]]."""
    return np.array([[b, a], [-a, b]], dtype=object)


def tilt_forward(w: np.ndarray, a: int, b: int) -> np.ndarray:
    """y = U^T w = (b w_1 - a w_2, a w_1 + b w_2) (eq. (21) times c)."""
    w = np.asarray(w, dtype=np.int64)
    return np.stack([b * w[:, 0] - a * w[:, 1], a * w[:, 0] + b * w[:, 1]], axis=1)


def tilt_back(y: np.ndarray, a: int, b: int, c: int, N: int):
    """w = U y / c^2, and whether each row is an image of [-N/2, N/2)^2 (divisible by
    c^2, inside the box)."""
    y = np.asarray(y, dtype=np.int64)
    u = np.stack([b * y[:, 0] + a * y[:, 1], -a * y[:, 0] + b * y[:, 1]], axis=1)
    c2 = int(c) * int(c)
    ok = np.all(u % c2 == 0, axis=1)
    w = u // c2
    ok &= np.all((w >= -(N // 2)) & (w < N // 2), axis=1)
    return w, ok


def tilt_range(N: int, a: int, b: int) -> list[tuple[int, int]]:
    """Inclusive range of each rotated coordinate over w in [-N/2, N/2)^2."""
    lo_w, hi_w = -(N // 2), N // 2 - 1
    return [(b * lo_w - a * hi_w, b * hi_w - a * lo_w), ((a + b) * lo_w, (a + b) * hi_w)]
