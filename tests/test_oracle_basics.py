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
