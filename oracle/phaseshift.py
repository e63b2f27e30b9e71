"""Phaseshift, the 1-D algorithm of Section 2.1 (its listing), in FP64.

Two sample sets of length p per round, f(h/p) and f(h/p + eps) (eq. (2),
reading R1 of the MultiPhaseshift module), their DFTs, the test of eq. (8)
and the decode of eq. (7):  w = Arg(F_eps[h] / F_0[h]) / (2 pi eps),
a = F_0[h] / p.  Adaptive: g built from R is subtracted from the samples.
"""
from __future__ import annotations

import math

import numpy as np

from .transforms import dft
from .philox import sample_noise
from .primes import ith_prime_at_least


def phaseshift_1d(freqs, coeffs, k: int, N: int, c: float = 5.0, eps: float | None = None,
                  tau: float | None = None, eta: float = 1e-3, max_rounds: int = 64,
                  sigma: float = 0.0, seed: int = 0, signal: int = 0):
    """Returns (w int64[kf] ascending, a complex128[kf], trace)."""
    w_pl = np.asarray(freqs, dtype=np.float64).reshape(-1)
    a_pl = np.asarray(coeffs, dtype=np.complex128)
    eps = 1.0 / (2.0 * N) if eps is None else eps
    tau = eps if tau is None else tau
    R: dict = {}
    trace = []
    i = 1
    while len(R) < k and i <= max_rounds:
        kstar = k - len(R)
        p = ith_prime_at_least(math.ceil(c * kstar), i)
        h = np.arange(p)
        t0 = h / p
        f = lambda t: np.exp(2j * np.pi * np.outer(t, w_pl)) @ a_pl
        v0 = f(t0) + sample_noise(seed, signal, i, 0, h, sigma)
        ve = f(t0 + eps) + sample_noise(seed, signal, i, 1, h, sigma)
        if R:
            wR = np.array(list(R.keys()), dtype=np.float64)
            aR = np.array(list(R.values()), dtype=np.complex128)
            v0 = v0 - np.exp(2j * np.pi * np.outer(t0, wR)) @ aR
            ve = ve - np.exp(2j * np.pi * (np.outer(t0, wR) + eps * wR[None, :])) @ aR
        F0, Fe = dft(v0), dft(ve)
        order = np.argsort(-np.abs(F0), kind="stable")[:kstar]
        cand = sorted(int(x) for x in order if abs(F0[x]) / p >= eta)
        acc = []
        for hb in cand:
            r = complex(Fe[hb]) / complex(F0[hb])
            if abs(abs(r) - 1.0) < tau:                       # eq. (8)
                th = math.atan2(r.imag, r.real)
                th = -math.pi if th >= math.pi else th
                x = th / (2.0 * math.pi * eps)                # eq. (7)
                wv = int(math.copysign(math.floor(abs(x) + 0.5), x))
                acc.append((wv, complex(F0[hb]) / p))
        for wv, a in acc:
            R[wv] = R.get(wv, 0.0) + a
        R = {wv: a for wv, a in R.items() if abs(a) >= eta}
        trace.append(dict(i=i, kstar=kstar, p=p, m=1, n_cand=len(cand), n_acc=len(acc),
                          n_R=len(R)))
        i += 1
    ws = np.array(sorted(R.keys()), dtype=np.int64)
    return ws, np.array([R[int(x)] for x in ws], dtype=np.complex128), trace
