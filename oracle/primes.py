"""Prime choice of the method (oracle side).

Algorithm MultiPhaseshift (Section 4.1.2) sets p to the i-th prime number
that is at least c k* in round i (the same rule appears in Algorithms
Phaseshift and 2DTiltedPhaseshift).  Section 5.0 words it as "the next larger
prime"; the oracle takes the literal i-th-prime reading, which keeps p
changing between rounds even when k* stalls.

The "smooth" variant restricts the choice to primes p whose p - 1 has no
prime factor above 7 (a plan option, not in the paper).
"""
from __future__ import annotations

import math


def is_prime(n: int) -> bool:
    """Trial division: plain and obviously correct."""
    n = int(n)
    if n < 2:
        return False
    if n < 4:
        return True
    if n % 2 == 0:
        return False
    r = math.isqrt(n)
    f = 3
    while f <= r:
        if n % f == 0:
            return False
        f += 2
    return True


def is_7smooth(n: int) -> bool:
    n = int(n)
    if n < 1:
        return False
    for f in (2, 3, 5, 7):
        while n % f == 0:
            n //= f
    return n == 1


def primes_upto(n: int) -> list[int]:
    return [q for q in range(2, int(n) + 1) if is_prime(q)]


def ith_prime_at_least(x: int, i: int, smooth: bool = False) -> int:
    """The i-th (1-based) prime q >= x; with `smooth`, only primes with 7-smooth q - 1."""
    if i < 1:
        raise ValueError("i is 1-based")
    q = max(2, int(x))
    seen = 0
    while True:
        if is_prime(q) and (not smooth or is_7smooth(q - 1)):
            seen += 1
            if seen == i:
                return q
        q += 1
