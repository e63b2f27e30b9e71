"""MultiPhaseshift (Section 4.1.2 listing, explained in Section 5.0), in FP64.

One call recovers one signal.  Round i (1-based):

  k*  = k - |R|                                         (listing; Section 5.0)
  p   = i-th prime >= c k*                             (listing; prime rule)
  m   = (i mod d2) + 1                                 (listing; projection axis)
  sets: s = 0 unshifted; s = 1..d2 shifted by eps along unwrapped axis n = s;
        with a ladder K > 1 also s = d2+1..2 d2 shifted by K eps along n = s - d2
  v_s[h] = f(t_h) - g(t~_h),  t_h = (h/p) U e_m + eps_s U e_n   (eqs. (36), (41))
           g(t~) = sum_{(y, a) in R} a exp(2 pi i y . t~)      (adaptive residual,
                                                               Section 5.0)
  F_s = DFT(v_s)                                               (Section 2.1)
  candidates: the k* buckets of largest |F_0| (sorted, Section 5.0)
  test:   | |F_s[h]| / |F_0[h]| - 1 | < tau  for every shifted set (eq. (42))
  decode: y_n = Arg(F_n[h] / F_0[h]) / (2 pi eps),  a = F_0[h] / p   (eq. (41))
  R <- R u {(y, a)};  prune small coefficients;  i <- i + 1
  finally wrap each y back to w (inverse of eq. (35))

The readings taken where the paper is silent or inconsistent are listed in
READINGS and cited in the code by their key.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .transforms import dft
from .philox import sample_noise
from .primes import ith_prime_at_least
from .signal import evaluate, sample_points
from .classifier import bf16_round, bucket_features, bucket_label, prob_single
from .unwrapping import (partition, pythagorean_tilt, tilt_back, tilt_forward, tilt_range,
                         unwrap, unwrap_matrix, wrap, y_range)

READINGS = {
    "R1": "Phaseshift listing labels the shifted and unshifted sample vectors the other "
          "way round from eq. (2); the eps-labelled set is the shifted one.",
    "R2": "Sample index h runs over 0..p-1 at h/p (eq. (2)); the listings' (h-1)/p, h=1..p "
          "is the same point set.",
    "R3": "Unwrapping powers are N^0..N^(d1-1) (eq. (35)); the sampling line of the listing "
          "writes N^1..N^d1.",
    "R4": "Block of coordinate l (1-based) is floor((l-1)/d1)+1, consistent with eq. (38).",
    "R5": "Collision ratio is |F_shifted| / |F_0| as in eqs. (8), (42) (the listings invert "
          "it; the test is symmetric to first order).",
    "R6": "Test tolerance tau is a parameter; the listing compares against eps, which is the "
          "default.  Noisy inputs add tau_noise*sqrt(p)/|F_0[h]| (not in the paper).",
    "R7": "SORT orders buckets by |F_0| descending, ties by ascending h; the first k* are "
          "tested; the same permutation applies to every shifted set.",
    "R8": "'Prune small coefficients' drops |a| < eta; buckets with |F_0[h]|/p < eta are "
          "not candidates.",
    "R9": "p is the i-th prime >= max(ceil(c k*), p_min) in round i (p_min = 0 is the "
          "paper's rule; the smooth rule keeps primes with 7-smooth p-1).",
    "R10": "R is a map from y to a; accepting an existing y adds the coefficients, in "
           "ascending bucket order.",
    "R11": "Decoded frequencies are rounded to the nearest integer, ties away from zero.",
    "R12": "Arg takes values in [-pi, pi): atan2's +pi maps to -pi.",
    "R13": "The loop also stops after max_rounds rounds (status NOT_CONVERGED).",
    "R15": "The unshifted set does not depend on n (eq. (41)) and is sampled once per round.",
    "R16": "A decoded coordinate outside the unwrapped band [-(N/2) S, (N/2-1) S], "
           "S = sum N^r, cannot be a frequency of the signal model (eq. (32)) and the bucket "
           "is rejected.",
    "R17": "Robust mode (not in the paper): also reject a bucket unless y_m = h (mod p) and "
           "the coarse decode lies within N^d1/(4K) of the ladder-refined one.",
    "R18": "Noise ladder (not in the paper): with K > 1 each axis also gets a K eps shift; "
           "y = y_c + round(wrap(theta_K - 2 pi K eps y_c) / (2 pi K eps)).",
    "R21": "Learned classifier (not in the paper): accept iff the network's singleton "
           "probability on the 8 bucket features exceeds a threshold and the decode is valid; "
           "the plain ratio test of eq. (42) is the fallback.",
    "R14": "Verification (not in the paper, which stops at |R| = k): when |R| reaches k, "
           "round i samples the residual once along the tilted line t_h = (h/p) U v, "
           "v_n = q^(n-1) mod p, q = 1 + (i mod (p-1)), p the round's prime for k* = 1 "
           "(every unwrapped coordinate enters the bucket index, so residual modes rarely "
           "share a bucket), and transforms it; if some bucket has |F[h]|/p >= verify_eta "
           "the next round runs with k* = min(that count, k, k + max(16, ceil(k/8)) - |R|), "
           "so the registry never exceeds k + max(16, ceil(k/8)) entries; when that is 0, or "
           "the round cap ends the loop before a clean check, or |R| > k at the end, the "
           "status is RESIDUAL_NONZERO.",
    "R19": "Noise (not in the paper): sigma/sqrt(2) (g1 + i g2) per sample from "
           "Philox4x64-10, key (seed, signal), counter (h // 2, set, round, 0), output "
           "words 0, 1 for even h and 2, 3 for odd h.",
    "R22": "General partitions (Section 4.1 on the free order of a block's coordinates and "
           "blocks of different sizes; Section 4.1.2 on prime d): blocks of sizes d_q "
           "(sum d) over a coordinate order pi, y_q = sum_r w_{pi(s_q + r)} N^r with s_q the "
           "block's first position; one shift eps = 1/(2 N^max d_q) on every axis, below the "
           "inverse of the largest block bandwidth as the paper chooses (not one eps per "
           "block); the band check of R16 uses each coordinate's own block size.",
    "R23": "2D tilting (Section 3.3, Theorem 1): for d = 2 the whole recovery runs on lines "
           "t = U t~, U = [[b, a], [-a, b]] (eq. (27): rotation by sin = a/c, cos = b/c scaled "
           "by c), y = U^T w, and w = U y / c^2 at the end (the listing's rotation back, "
           "exact in integers).  (a, b, c) is a Pythagorean triple with b > 2N and "
           "gcd(a, b) = 1; unless given, the one with the smallest bandwidth a + b.  "
           "eps = 1/(2 NB), NB = (a + b) N / 2 bounds every rotated coordinate.  A decoded "
           "y is no mode unless U y is divisible by c^2 with the quotient in [-N/2, N/2)^2 "
           "(the rotated form of R16).",
}

STATUS_OK = 0
STATUS_NOT_CONVERGED = 1
STATUS_RESIDUAL_NONZERO = 2


@dataclass
class Params:
    d: int
    N: int
    k: int
    d1: int = 1
    blocks: tuple | None = None        # R22: block sizes (sum d); None = uniform d1
    order: tuple | None = None         # R22: coordinate order; None = natural
    tilt: object = None                # R23 (d = 2): None, True (triple of Theorem 1) or (a, b, c)
    c: float = 5.0
    ladder_K: int = 1
    tau: float | None = None
    tau_noise: float = 0.0
    eta: float = 1e-3
    max_rounds: int = 64
    prime_rule: str = "paper"
    p_min: int = 0
    robust: bool = False
    classifier: str = "plain"          # "plain" (eq. (42)) or "mlp" (R21)
    mlp_params: np.ndarray | None = None
    mlp_threshold: float = 0.5
    feature_scale: float | None = None  # None: tau_eff
    verify: bool = False               # R14
    verify_eta: float | None = None    # None: eta

    @property
    def block_sizes(self) -> tuple:
        """Size of each unwrapped block (d2 entries)."""
        return partition(self.d, self.d1, self.blocks, self.order)[0]

    @property
    def tilt_abc(self):
        """(a, b, c) of the rotation (R23), or None."""
        if self.tilt is None or self.tilt is False:
            return None
        if self.tilt is True:
            return pythagorean_tilt(int(self.N))
        return tuple(int(v) for v in self.tilt)

    @property
    def d2(self) -> int:
        return 2 if self.tilt_abc else len(self.block_sizes)

    @property
    def NB(self) -> int:
        """Largest bandwidth of an unwrapped coordinate, N^d1 (R22: N^max d_q; R23:
        (a + b) N / 2, which bounds every rotated coordinate)."""
        t = self.tilt_abc
        if t:
            return (t[0] + t[1]) * int(self.N) // 2
        return int(self.N) ** max(self.block_sizes)

    def line_matrix(self) -> np.ndarray:
        """U of the sampling lines, t = U t~ (eq. (36); eq. (27) when tilted)."""
        return unwrap_matrix(self.d, self.d1, self.N, self.blocks, self.order, self.tilt_abc)

    def to_lines(self, w) -> np.ndarray:
        """y = U^T w."""
        t = self.tilt_abc
        if t:
            return tilt_forward(w, t[0], t[1])
        return unwrap(w, self.d1, self.N, self.blocks, self.order)

    def from_lines(self, y) -> np.ndarray:
        """w from y (the inverse of to_lines on its image)."""
        t = self.tilt_abc
        if t:
            w, ok = tilt_back(y, t[0], t[1], t[2], int(self.N))
            if not np.all(ok):
                raise ValueError("value outside the rotated image")
            return w
        return wrap(y, self.d1, self.N, self.blocks, self.order)

    def bands(self) -> list:
        """Inclusive range of each unwrapped coordinate (R16)."""
        t = self.tilt_abc
        if t:
            return tilt_range(int(self.N), t[0], t[1])
        return [y_range(self.N, dn) for dn in self.block_sizes]

    def in_image(self, y) -> bool:
        """Whether y = U^T w for some w in [-N/2, N/2)^d (R16, R23)."""
        t = self.tilt_abc
        if t:
            return bool(tilt_back(np.asarray(y, np.int64)[None, :], t[0], t[1], t[2],
                                  int(self.N))[1][0])
        return all(lo <= int(v) <= hi for v, (lo, hi) in zip(y, self.bands()))

    @property
    def eps(self) -> float:
        """Shift eps = 1 / (2 N^d1) (Section 5); one eps for every axis (R22)."""
        return 1.0 / (2.0 * self.NB)

    @property
    def tau_eff(self) -> float:
        return self.eps if self.tau is None else float(self.tau)

    def validate(self):
        if self.d < 1:
            raise ValueError("d must be positive")
        partition(self.d, self.d1, self.blocks, self.order)  # raises on a bad partition
        t = self.tilt_abc
        if t:
            a, b, c = t
            if self.d != 2 or self.blocks is not None or self.order is not None or self.d1 != 1:
                raise ValueError("tilting is defined for d = 2 without unwrapping")
            if not (1 <= a < b < c and a * a + b * b == c * c and math.gcd(a, b) == 1
                    and b > 2 * self.N):
                raise ValueError("the tilt must be a Pythagorean triple with b > 2N, gcd(a, b) = 1")
        if self.N < 2 or self.N % 2:
            raise ValueError("N must be even and >= 2")
        if self.k < 1 or self.c <= 1.0 or self.ladder_K < 1:
            raise ValueError("bad k, c or ladder_K")


def shift_table(d2: int, ladder_K: int):
    """[(n, K)] for sets s = 1..S: coarse eps on each axis, then K eps on each axis."""
    tab = [(n, 1) for n in range(1, d2 + 1)]
    if ladder_K > 1:
        tab += [(n, int(ladder_K)) for n in range(1, d2 + 1)]
    return tab


@dataclass
class Result:
    freqs: np.ndarray          # int64 [kf, d], lexicographic order
    coeffs: np.ndarray         # complex128 [kf]
    y: np.ndarray              # int64 [kf, d2] unwrapped, same order
    status: int
    rounds: int
    samples: int
    trace: list = field(default_factory=list)
    spectra: list = field(default_factory=list)
    registry: list = field(default_factory=list)


def _round_half_away(x: float) -> int:
    """R11."""
    return int(math.copysign(math.floor(abs(x) + 0.5), x))


def _arg(z: complex) -> float:
    """R12: Arg in [-pi, pi)."""
    th = math.atan2(z.imag, z.real)
    return -math.pi if th >= math.pi else th


def _wrap_pi(x: float) -> float:
    return x - 2.0 * math.pi * math.floor((x + math.pi) / (2.0 * math.pi))


def _residual(yR, aR, p, m, n, shift):
    """g(t~_h) = sum_{(y, a) in R} a exp(2 pi i ((h/p) y_m + shift y_n)) for h = 0..p-1."""
    h = np.arange(p, dtype=np.float64)
    ph = np.outer(h / p, yR[:, m - 1].astype(np.float64))
    ph = ph + shift * yR[:, n - 1].astype(np.float64)[None, :]
    return np.exp(2j * np.pi * ph) @ aR


def verify_samples(freqs, coeffs, P: Params, p: int, q: int, i: int, yR, aR,
                   sigma: float = 0.0, seed: int = 0, signal: int = 0) -> np.ndarray:
    """R14: residual samples f(t_h) + noise - g(t_h) on the tilted line
    t_h = (h/p) U v, v_n = q^(n-1) mod p, h = 0..p-1 (noise of set 0, round i)."""
    v = np.array([pow(int(q), n, int(p)) for n in range(P.d2)], dtype=np.int64)
    direction = P.line_matrix().astype(np.float64) @ v.astype(np.float64)
    h = np.arange(p)
    t = (h.astype(np.float64) / p)[:, None] * direction[None, :]
    out = evaluate(freqs, coeffs, t) + sample_noise(seed, signal, i, 0, h, sigma)
    if len(aR):
        ph = np.outer(h.astype(np.float64) / p, (np.asarray(yR) @ v).astype(np.float64))
        out = out - np.exp(2j * np.pi * ph) @ np.asarray(aR)
    return out


def _plain_test(F, h, p, P: Params) -> bool:
    """eq. (42): | |F_s[h]| / |F_0[h]| - 1 | < tau for every shifted set (R5, R6)."""
    F0 = complex(F[0][h])
    thr = P.tau_eff + (P.tau_noise * math.sqrt(p) / abs(F0) if P.tau_noise > 0 else 0.0)
    for s in range(1, len(F)):
        if not abs(abs(complex(F[s][h]) / F0) - 1.0) < thr:
            return False
    return True


def _test_margin(F, h, p, P: Params) -> float:
    """Distance of bucket h's ratio test (eq. (42)) from its threshold, in units of the
    ratio: min over the shifted sets of | thr - | |F_s/F_0| - 1 | |.  A diagnostic of how
    near a tie the decision was; it decides nothing."""
    F0 = complex(F[0][h])
    thr = P.tau_eff + (P.tau_noise * math.sqrt(p) / abs(F0) if P.tau_noise > 0 else 0.0)
    return min(abs(thr - abs(abs(complex(F[s][h]) / F0) - 1.0)) for s in range(1, len(F)))


def _select_margin(absF0, order, kstar: int, p: int, eta: float) -> float:
    """Distance of the candidate choice (R7, R8) from a tie, in units of |F_0|/p (a
    coefficient): the gap between the k*-th and (k*+1)-th largest |F_0| when that cut
    decides between candidates, and the distance of each chosen |F_0|/p from the floor
    eta.  Diagnostic only."""
    m = math.inf
    if kstar < len(absF0):
        a, b = absF0[order[kstar - 1]], absF0[order[kstar]]
        if max(a, b) / p >= eta:          # the order at the cut changes the candidates
            m = min(m, (a - b) / p)
    for x in order[:kstar]:
        m = min(m, abs(absF0[x] / p - eta))
    return m


def _decode(F, h, p, m, P: Params):
    """Phase-ratio decode of eq. (41) with the ladder (R18); returns (y, valid).

    valid: every coordinate in band (R16) and, in robust mode, the residue and
    ladder-consistency checks (R17).
    """
    F0 = complex(F[0][h])
    NB = P.NB
    valid = True
    y = np.zeros(P.d2, dtype=np.int64)
    for n in range(1, P.d2 + 1):
        th = _arg(complex(F[n][h]) / F0)
        yc_real = th * NB / math.pi            # Arg / (2 pi eps) with eps = 1/(2 NB)
        yn = _round_half_away(yc_real)
        if P.ladder_K > 1:                     # R18
            K = P.ladder_K
            thf = _arg(complex(F[P.d2 + n][h]) / F0)
            q = (K * yn) % (2 * NB)            # 2 pi K eps yn, reduced exactly
            delta = _wrap_pi(thf - math.pi * q / NB)
            yn = yn + _round_half_away(delta * NB / (math.pi * K))
            if P.robust and abs(yc_real - yn) > NB / (4.0 * K):
                valid = False
        y[n - 1] = yn
    if not P.in_image(y):                      # R16 (R23: and the rotated lattice)
        valid = False
    if P.robust and (int(y[m - 1]) % p) != h:  # R17
        valid = False
    return y, valid


def _coefficient(F0h, p: int) -> complex:
    """a = F_0[h] / p (eq. (41))."""
    return complex(F0h) / p


def _features(F, h, y, m, P: Params) -> np.ndarray:
    scale = P.tau_eff if P.feature_scale is None else P.feature_scale
    return bucket_features(F, h, y, m, P.d2, P.ladder_K, P.NB, scale)


def round_samples(freqs, coeffs, P: Params, p: int, m: int, i: int, yR, aR,
                  sigma: float = 0.0, seed: int = 0, signal: int = 0,
                  hs=None) -> np.ndarray:
    """The S+1 sample sets of round i: v_s[h] = f(t_h) + noise - g(t~_h), complex [S+1, p].

    t_h = (h/p) U e_m + eps_s U e_n (eqs. (36), (41)); g is the registry
    {(yR[e], aR[e])} evaluated on the unwrapped line (Section 5.0).  Set 0 is
    unshifted and is sampled once per round (R15).  hs: only these points h
    (columns of the result, in the given order); default all p.
    """
    d, d1, N = P.d, P.d1, P.N
    tab = shift_table(P.d2, P.ladder_K)
    h = np.arange(p) if hs is None else np.asarray(hs, dtype=np.int64)
    V = []
    for s, (n, K) in enumerate([(1, 0)] + tab):
        shift = P.eps * K
        t = sample_points(d, d1, N, p, m, n, shift, P.blocks, P.order, P.tilt_abc)[h]
        v = evaluate(freqs, coeffs, t)
        v = v + sample_noise(seed, signal, i, s, h, sigma)
        if len(aR):                                        # adaptive subtraction of g
            v = v - _residual(np.asarray(yR), np.asarray(aR), p, m, n, shift)[h]
        V.append(v)
    return np.array(V)


def multiphaseshift(freqs, coeffs, P: Params, sigma: float = 0.0, seed: int = 0,
                    signal: int = 0, keep_spectra: bool = False, collect: list | None = None
                    ) -> Result:
    """Recover the spectrum of the planted signal sum_j coeffs[j] e^{2 pi i freqs[j] . t}.

    The signal is only evaluated as a black box at the sampling points; the
    planted lists are never read otherwise.
    """
    P.validate()
    freqs = np.asarray(freqs, dtype=np.int64)
    coeffs = np.asarray(coeffs, dtype=np.complex128)
    d, d1, d2, N = P.d, P.d1, P.d2, P.N
    y_planted = P.to_lines(freqs) if collect is not None else None
    tab = shift_table(d2, P.ladder_K)
    R: dict = {}
    trace, spectra, registry = [], [], []
    samples = 0
    i = 1
    k_next = 0          # k* of the round after a verification that found residual energy
    verified = False
    smooth = P.prime_rule == "smooth"
    while i <= P.max_rounds:                               # R13
        if len(R) >= P.k and k_next == 0:
            if not P.verify or verified:
                break
            # R14: is the residual empty?  One tilted line, prime for k* = 1.
            p = ith_prime_at_least(max(math.ceil(P.c), P.p_min), i, smooth=smooth)
            q = 1 + (i % (p - 1))
            yR = np.array(list(R.keys()), dtype=np.int64).reshape(-1, d2)
            aR = np.array(list(R.values()), dtype=np.complex128)
            F0 = dft(verify_samples(freqs, coeffs, P, p, q, i, yR, aR, sigma=sigma,
                                    seed=seed, signal=signal))
            samples += p
            veta = P.eta if P.verify_eta is None else P.verify_eta
            n_res = int(np.count_nonzero(np.abs(F0) / p >= veta))
            vmargin = float(np.min(np.abs(np.abs(F0) / p - veta)))
            trace.append(dict(i=i, kstar=0, p=p, m=0, n_cand=n_res, n_acc=0, n_R=len(R),
                              verify=1, margin_ratio=math.inf, margin_coeff=vmargin))
            i += 1
            if n_res == 0:
                verified = True
                continue
            # the registry may grow past k by at most `extra` entries while it is repaired
            extra = max(16, math.ceil(P.k / 8))
            k_next = min(n_res, P.k, P.k + extra - len(R))
            if k_next <= 0:
                break
            continue
        kstar = P.k - len(R) if len(R) < P.k else k_next
        k_next = 0
        p = ith_prime_at_least(max(math.ceil(P.c * kstar), P.p_min), i, smooth=smooth)
        m = (i % d2) + 1
        snapshot = (np.array(list(R.keys()), dtype=np.int64).reshape(-1, d2),
                    np.array(list(R.values()), dtype=np.complex128))
        V = round_samples(freqs, coeffs, P, p, m, i, snapshot[0], snapshot[1],
                          sigma=sigma, seed=seed, signal=signal)
        F = [dft(v) for v in V]
        samples += len(F) * p
        F0 = F[0]
        full_order = np.argsort(-np.abs(F0), kind="stable")
        order = full_order[:kstar]                                       # R7
        cand = sorted(int(x) for x in order if abs(F0[x]) / p >= P.eta)  # R8
        margin_coeff = _select_margin(np.abs(F0), full_order, kstar, p, P.eta)
        margin_ratio = math.inf
        accepted = []
        for hb in cand:
            y, valid = _decode(F, hb, p, m, P)
            if P.classifier == "mlp" or collect is not None:
                feats = _features(F, hb, y, m, P)
            if P.classifier == "mlp":
                x = bf16_round(feats)
                ok = valid and prob_single(P.mlp_params, x[None, :])[0] > P.mlp_threshold
            else:
                ok = valid and _plain_test(F, hb, p, P)
                if valid:
                    margin_ratio = min(margin_ratio, _test_margin(F, hb, p, P))
            if collect is not None:
                collect.append((i, hb, feats, bucket_label(hb, p, m, y_planted, coeffs, R, P.eta),
                                int(ok), abs(F0[hb]) / p))
            if ok:
                accepted.append((tuple(int(v) for v in y), _coefficient(F0[hb], p)))
        for y, a in accepted:                                            # R10
            R[y] = R.get(y, 0.0) + a
        R = {y: a for y, a in R.items() if abs(a) >= P.eta}              # R8
        trace.append(dict(i=i, kstar=kstar, p=p, m=m, n_cand=len(cand),
                          n_acc=len(accepted), n_R=len(R), verify=0,
                          margin_ratio=margin_ratio, margin_coeff=margin_coeff))
        if keep_spectra:
            spectra.append(np.array(F))
            registry.append(snapshot)
        i += 1
    if len(R) < P.k:
        status = STATUS_NOT_CONVERGED
    elif len(R) > P.k or (P.verify and not verified):
        status = STATUS_RESIDUAL_NONZERO
    else:
        status = STATUS_OK
    if R:
        ys = np.array(list(R.keys()), dtype=np.int64).reshape(-1, d2)
        a = np.array(list(R.values()), dtype=np.complex128)
        w = P.from_lines(ys)
        order = np.lexsort(w.T[::-1])
        w, a, ys = w[order], a[order], ys[order]
    else:
        w = np.zeros((0, d), np.int64)
        a = np.zeros(0, np.complex128)
        ys = np.zeros((0, d2), np.int64)
    return Result(freqs=w, coeffs=a, y=ys, status=status, rounds=i - 1,
                  samples=samples, trace=trace, spectra=spectra,
                  registry=registry)
