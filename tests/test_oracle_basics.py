"""Pins of the oracle's building blocks against things other than the oracle.

Primes against the prime-counting function, unwrapping against exhaustive
enumeration, Philox against its published known-answer vector and numpy's
independent implementation, the DFT against its O(M^2) definition, and the
sampled spectra against the closed form of eqs. (3) and (41).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import philox
from oracle import unwrapping as uw

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_prime_counting():
    # pi(10^4) = 1229 and pi(10^3) = 168 (textbook values)
    assert len(oracle.primes_upto(10000)) == 1229
    assert len(oracle.primes_upto(1000)) == 168
    assert not oracle.is_prime(1) and oracle.is_prime(2) and not oracle.is_prime(3001 * 3)


def test_ith_prime_rule():
    # i-th prime >= x, 1-based (listing's prime rule)
    assert oracle.ith_prime_at_least(40, 1) == 41
    assert oracle.ith_prime_at_least(40, 2) == 43
    assert oracle.ith_prime_at_least(3000, 1) == 3001
    assert oracle.ith_prime_at_least(15, 2) == 19
    assert oracle.ith_prime_at_least(13, 1) == 13
    # smooth rule: p - 1 has only factors 2, 3, 5, 7 (3001 - 1 = 2^3 3 5^3)
    q = oracle.ith_prime_at_least(2000, 1, smooth=True)
    assert q == 2017 and 2016 == 2 ** 5 * 3 ** 2 * 7


@pytest.mark.parametrize("N,d1", [(4, 3), (20, 2), (64, 2), (6, 2), (2, 5)])
def test_unwrap_bijection_exhaustive(N, d1):
    # every digit vector in [-N/2, N/2)^d1 -> distinct y, covering a range of N^d1 integers
    grids = np.meshgrid(*[np.arange(-N // 2, N // 2)] * d1, indexing="ij")
    w = np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.int64)
    y = uw.unwrap(w, d1, N)
    assert len(np.unique(y)) == N ** d1
    lo, hi = uw.y_range(N, d1)
    assert y.min() == lo and y.max() == hi and hi - lo + 1 == N ** d1
    assert np.array_equal(uw.wrap(y, d1, N), w)
    # eq. (35) written out for the first digit vector
    assert y[0, 0] == sum((-N // 2) * N ** r for r in range(d1))


@pytest.mark.parametrize("N,blocks,order", [(4, (2, 3), (4, 0, 3, 1, 2)), (6, (1, 2), (1, 2, 0)),
                                            (20, (3, 1), None), (2, (1, 4, 2), (6, 5, 4, 3, 2, 1, 0))])
def test_unwrap_general_bijection_exhaustive(N, blocks, order):
    # a general partition maps [-N/2, N/2)^d one to one onto the product of its blocks' bands
    d = sum(blocks)
    grids = np.meshgrid(*[np.arange(-N // 2, N // 2)] * d, indexing="ij")
    w = np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.int64)
    y = uw.unwrap(w, 1, N, blocks, order)
    assert y.shape == (N ** d, len(blocks))
    assert len(np.unique(y, axis=0)) == N ** d
    for q, dq in enumerate(blocks):
        lo, hi = uw.y_range(N, dq)
        assert y[:, q].min() == lo and y[:, q].max() == hi
    assert np.array_equal(uw.wrap(y, 1, N, blocks, order), w)
    U = uw.unwrap_matrix(d, 1, N, blocks, order)
    assert np.array_equal((w.astype(object) @ U).astype(np.int64), y)


def test_unwrap_general_by_hand():
    # d = 3, blocks (2, 1), order (2, 0, 1): y_0 = w_2 + N w_0, y_1 = w_1
    y = uw.unwrap(np.array([[1, -2, 3]]), 1, 8, (2, 1), (2, 0, 1))
    assert y.tolist() == [[3 + 8 * 1, -2]]
    # the paper's uneven split of its 20-dimensional example: four blocks of 3, two of 4
    P = oracle.Params(d=20, N=20, k=1, blocks=(3, 3, 3, 3, 4, 4))
    assert P.d2 == 6 and P.NB == 20 ** 4 and P.eps == 1.0 / 320000.0
    lo, hi = uw.y_range(20, 3)
    assert hi - lo + 1 == 8000
    for bad in [dict(blocks=(3, 3)), dict(blocks=(0, 20)), dict(order=tuple(range(19)) + (0,))]:
        with pytest.raises(ValueError):
            oracle.Params(d=20, N=20, k=1, **bad).validate()


@pytest.mark.parametrize("N", [4, 8, 16, 20, 64])
def test_pythagorean_tilt_is_smallest(N):
    # brute force over all integer legs: the plan's triple satisfies Theorem 1 (b > 2N,
    # gcd(a, b) = 1, c > b > a) with the smallest bandwidth a + b
    best = None
    for b in range(2 * N + 1, 8 * N + 1):
        for a in range(1, b):
            c2 = a * a + b * b
            c = math.isqrt(c2)
            if c * c == c2 and math.gcd(a, b) == 1:
                key = (a + b, b)
                if best is None or key < best[0]:
                    best = (key, (a, b, c))
    assert uw.pythagorean_tilt(N) == best[1]


def test_tilt_theorem_no_collisions():
    # Theorem 1, exhaustively at N = 16: no two frequencies share a rotated coordinate,
    # the rotation back is exact, and the bands are the extremes of the image
    N = 16
    a, b, c = uw.pythagorean_tilt(N)
    g = np.arange(-N // 2, N // 2)
    w = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2).astype(np.int64)
    y = uw.tilt_forward(w, a, b)
    assert len(np.unique(y[:, 0])) == N * N and len(np.unique(y[:, 1])) == N * N
    back, ok = uw.tilt_back(y, a, b, c, N)
    assert ok.all() and np.array_equal(back, w)
    for shift in ((1, 0), (0, 1), (c, 0)):
        assert not uw.tilt_back(y + np.array(shift), a, b, c, N)[1].any()
    for q, (lo, hi) in enumerate(uw.tilt_range(N, a, b)):
        assert y[:, q].min() == lo and y[:, q].max() == hi
    # the condition b > 2N matters: the (3, 4, 5) rotation leaves collisions at N = 16
    y345 = uw.tilt_forward(w, 3, 4)
    assert len(np.unique(y345[:, 0])) < N * N
    # y = U^T w with U of eq. (27): (b w_1 - a w_2, a w_1 + b w_2), by hand for one point
    assert uw.tilt_forward(np.array([[2, -3]]), a, b).tolist() == [[2 * b + 3 * a, 2 * a - 3 * b]]


def test_tilt_phase_identity():
    # f on the lines t = U t~ equals the signal with frequencies y = U^T w in t~ (eq. (27))
    rng = np.random.default_rng(5)
    N = 64
    a, b, c = uw.pythagorean_tilt(N)
    w = rng.integers(-N // 2, N // 2, size=(6, 2))
    amp = rng.normal(size=6) + 1j * rng.normal(size=6)
    tt = rng.uniform(-1, 1, size=(10, 2))
    U = uw.tilt_matrix(a, b).astype(float)
    lhs = oracle.evaluate(w, amp, tt @ U.T)
    rhs = oracle.evaluate(uw.tilt_forward(w, a, b), amp, tt)
    assert np.abs(lhs - rhs).max() < 1e-9


def test_unwrap_paper_example():
    ex = GOLD["worked_example"]
    lo, hi = uw.y_range(ex["N"], ex["d1"])
    assert hi - lo + 1 == ex["unwrapped_bandwidth"]
    lo5, hi5 = uw.y_range(20, 5)
    assert (lo5, hi5) == (-1684210, 1515789)
    P = oracle.Params(d=100, N=20, k=1, d1=5)
    assert P.d2 == 20 and P.eps == GOLD["section5_experiment"]["eps"]


def test_unwrap_phase_identity():
    # f evaluated on the unwrapped line t = U t~ equals the d2-dim signal with y = U^T w (eq. (38))
    rng = np.random.default_rng(1)
    d, d1, N = 6, 3, 8
    w = rng.integers(-N // 2, N // 2, size=(5, d))
    a = rng.normal(size=5) + 1j * rng.normal(size=5)
    tt = rng.uniform(size=(7, d // d1))
    U = uw.unwrap_matrix(d, d1, N).astype(float)
    lhs = oracle.evaluate(w, a, tt @ U.T)
    rhs = oracle.evaluate(uw.unwrap(w, d1, N), a, tt)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-10)


def test_philox_known_answer():
    kat = GOLD["philox4x64_10_kat"]
    out = philox.philox4x64_10([np.uint64(x) for x in kat["counter"]],
                               [np.uint64(x) for x in kat["key"]])
    assert [format(int(x), "016x") for x in out] == kat["out"]


def test_philox_matches_numpy():
    # numpy's Philox increments the 256-bit counter before producing each block
    key = np.array([0x0123456789ABCDEF, 0xFEDCBA9876543210], dtype=np.uint64)
    bg = np.random.Philox(key=key, counter=np.array([41, 7, 3, 0], dtype=np.uint64))
    ref = bg.random_raw(8).astype(np.uint64)
    for blk, c0 in enumerate((42, 43)):
        out = philox.philox4x64_10([np.uint64(c0), np.uint64(7), np.uint64(3), np.uint64(0)],
                                   [np.uint64(key[0]), np.uint64(key[1])])
        assert [int(x) for x in out] == [int(x) for x in ref[4 * blk:4 * blk + 4]]


def test_noise_statistics():
    h = np.arange(200000)
    n = philox.sample_noise(7, 3, 2, 5, h, sigma=0.25)
    assert abs(np.mean(n)) < 3 * 0.25 / math.sqrt(len(h))
    assert abs(np.mean(np.abs(n) ** 2) / 0.25 ** 2 - 1) < 0.02
    assert abs(np.mean(n.real * n.imag)) < 3 * 0.25 ** 2 / math.sqrt(len(h))
    # a different counter component gives a different stream
    n2 = philox.sample_noise(7, 3, 2, 6, h[:10], sigma=0.25)
    assert not np.allclose(n[:10], n2)
    assert np.array_equal(philox.sample_noise(7, 3, 2, 5, h[:10], 0.25), n[:10])


@pytest.mark.parametrize("M", [2, 3, 13, 41, 127, 1283])
def test_dft_definition(M):
    rng = np.random.default_rng(M)
    b = rng.normal(size=M) + 1j * rng.normal(size=M)
    assert np.allclose(oracle.dft(b), oracle.dft_direct(b), rtol=0, atol=1e-9 * M)
    # the DFT of one exponential e^{2 pi i x j / M} is M at bucket x and zero elsewhere
    x = M // 3
    e = np.exp(2j * np.pi * x * np.arange(M) / M)
    ref = np.zeros(M, complex)
    ref[x] = M
    assert np.allclose(oracle.dft(e), ref, atol=1e-9 * M)


@pytest.mark.parametrize("p,eps", [(13, 1 / 64), (41, 1 / 128), (101, 1e-3)])
def test_eq3_one_dim(p, eps):
    # eq. (3): F(f_{p,eps})[h] = p sum_{w = h mod p} a e^{2 pi i eps w}
    rng = np.random.default_rng(p)
    w = rng.choice(np.arange(-200, 200), size=20, replace=False)
    a = np.exp(2j * np.pi * rng.uniform(size=20))
    t = (np.arange(p) / p + eps)[:, None]
    F = oracle.dft(oracle.evaluate(w[:, None], a, t))
    ref = np.zeros(p, complex)
    for wj, aj in zip(w, a):
        ref[wj % p] += p * aj * np.exp(2j * np.pi * eps * wj)
    assert np.allclose(F, ref, atol=1e-9 * p)
