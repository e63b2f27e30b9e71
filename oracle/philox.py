"""Counter-based noise for the synthetic black-box signal.

The paper's method is noiseless (Section 1 and Section 6); the measured
configurations add complex Gaussian noise to every sample.  So that the oracle
and the HIP sampler see the same noise without passing it around, each side
implements Philox4x64-10 from its published definition (Salmon, Moraes,
Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC 2011):
ten rounds of two 64x64->128 multiplies with the round function

    (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))

and the key bumped by the Weyl constants (W0, W1) between rounds.

Noise of one sample (Box-Muller in FP64):
    key     = (seed, signal index)
    counter = (floor(h / 2), sample set, round, 0)
    u1, u2  = top 53 bits of output words 0 and 1 (even h) or 2 and 3 (odd h),
              times 2^-53
    g       = sqrt(-2 ln(1 - u1)) * (cos 2 pi u2 + i sin 2 pi u2)
    noise   = sigma / sqrt(2) * g        (so E|noise|^2 = sigma^2)
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, m: int):
    """(hi, lo) of the 128-bit product a * m, a uint64 array, m a constant."""
    a = a.astype(np.uint64)
    a_lo, a_hi = a & _MASK32, a >> _S32
    m_lo, m_hi = np.uint64(m & 0xFFFFFFFF), np.uint64(m >> 32)
    ll = a_lo * m_lo
    lh = a_lo * m_hi
    hl = a_hi * m_lo
    hh = a_hi * m_hi
    mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    with np.errstate(over="ignore"):
        lo = a * np.uint64(m)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds.  ctr: 4 uint64 arrays, key: 2 uint64 arrays."""
    c = [np.asarray(x, dtype=np.uint64) for x in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64)
    k1 = np.asarray(key[1], dtype=np.uint64)
    for r in range(10):
        if r:
            with np.errstate(over="ignore"):
                k0 = k0 + np.uint64(W0)
                k1 = k1 + np.uint64(W1)
        hi0, lo0 = _mulhilo(c[0], M0)
        hi1, lo1 = _mulhilo(c[2], M1)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def sample_noise(seed: int, signal: int, round_i: int, s: int, h: np.ndarray,
                 sigma: float) -> np.ndarray:
    """Complex noise added to samples h of set s in round round_i of one signal."""
    h = np.asarray(h, dtype=np.uint64)
    if sigma == 0.0:
        return np.zeros(h.shape, dtype=np.complex128)
    n = h.shape
    z = np.zeros(n, dtype=np.uint64)
    out = philox4x64_10(
        (h >> np.uint64(1), np.full(n, s, np.uint64), np.full(n, round_i, np.uint64), z),
        (np.full(n, np.uint64(seed & 0xFFFFFFFFFFFFFFFF)), np.full(n, signal, np.uint64)))
    odd = (h & np.uint64(1)).astype(bool)
    w0 = np.where(odd, out[2], out[0])
    w1 = np.where(odd, out[3], out[1])
    u1 = (w0 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u2 = (w1 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log1p(-u1))
    g = rad * (np.cos(2.0 * np.pi * u2) + 1j * np.sin(2.0 * np.pi * u2))
    return (sigma / np.sqrt(2.0)) * g
