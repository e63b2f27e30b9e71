"""Pins of oracle pieces that the paper does not fix and that other pins reach only
loosely: the noise-widened ratio test (reading R6), the Philox word layout of the
noise (reading R19) and the second feature axis n* of the learned classifier.

Each expected value is worked out by hand from a constructed input, so that a
plausible slip (p for sqrt(p), |F_0|^2 for |F_0|, even and odd samples swapped,
the radial and angular uniforms swapped, the axis picked by the coarse instead of
the fine ratio, ties to the larger axis) fails here.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import classifier as C
from oracle import method as M
from oracle import philox

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


# ----------------------------------------------------------- R6: tau_noise -----

def _spectra_with_ratios(F0, ratios, p):
    """S+1 spectra of length p whose bucket 0 has F_0[0] = F0 and F_s[0] / F_0[0] =
    ratios[s-1] exactly representable in FP64 (powers of two keep the quotient exact)."""
    F = np.zeros((len(ratios) + 1, p), dtype=np.complex128)
    F[0, 0] = F0
    for s, r in enumerate(ratios, start=1):
        F[s, 0] = F0 * r
    return F


@pytest.mark.parametrize("mag,tau_noise,want", [
    # |F_0| = 64, p = 4096: sqrt(p) / |F_0| = 1, so tau_noise adds tau_noise itself
    (1.0 + 2 ** -9, 0.0, False),        # 1.95e-3 off with tau = 1e-3: rejected
    (1.0 + 2 ** -9, 2 ** -10, True),    # threshold 1e-3 + 9.77e-4 = 1.98e-3 > 1.95e-3
    (1.0 + 2 ** -8, 2 ** -10, False),   # 3.9e-3 off: rejected even so
    (1.0 + 2 ** -8, 2 ** -8, True),     # threshold 1e-3 + 3.9e-3
])
def test_tau_noise_widens_ratio_test(mag, tau_noise, want):
    p, F0 = 4096, 64.0
    F = _spectra_with_ratios(F0, [1.0, mag, 1.0], p)
    P = oracle.Params(d=3, N=64, k=1, tau=1e-3, tau_noise=tau_noise)
    assert M._plain_test(F, 0, p, P) is want


def test_tau_noise_scales_with_sqrt_p_over_abs_f0():
    # the same relative deviation 2^-9 = 1.95e-3 and tau_noise = 2^-12 = 2.44e-4, tau = 1e-3:
    # |F_0| = 16, p = 4096 -> extra 2^-12 * 64 / 16 = 9.77e-4, threshold 1.98e-3: accepted;
    # |F_0| = 64 -> extra 2.44e-4: rejected; |F_0| = 16, p = 1024 -> extra 4.9e-4: rejected;
    # |F_0| = 16 at p = 16384 -> extra 1.95e-3: accepted
    dev = 1.0 + 2 ** -9
    P = oracle.Params(d=2, N=64, k=1, tau=1e-3, tau_noise=2 ** -12)
    cases = [(16.0, 4096, True), (64.0, 4096, False), (16.0, 1024, False), (16.0, 16384, True)]
    for F0, p, want in cases:
        F = _spectra_with_ratios(F0, [dev, 1.0], p)
        assert M._plain_test(F, 0, p, P) is want, (F0, p)
    # tau_noise = 0 is the paper's test: |F_0| and p play no part
    P0 = oracle.Params(d=2, N=64, k=1, tau=1e-3, tau_noise=0.0)
    for F0, p, _ in cases:
        assert M._plain_test(_spectra_with_ratios(F0, [dev, 1.0], p), 0, p, P0) is False
        assert M._plain_test(_spectra_with_ratios(F0, [1.0 + 2 ** -11, 1.0], p), 0, p, P0) is True


def test_tau_noise_changes_a_noisy_recovery():
    """On a noisy signal whose singletons miss tau = 1e-4 by the noise alone, the widened
    test accepts them in the first round (fewer rounds), with the same exact support."""
    import workloads
    w, a = workloads.planted_signal(3100, 0, 4, 1024, 40, (1.0, 2.0))
    base = dict(d=4, N=1024, k=40, c=3.0, ladder_K=64, tau=1e-4, eta=1e-3, p_min=101,
                robust=True, verify=True, verify_eta=1e-2, max_rounds=12)
    r0 = oracle.multiphaseshift(w, a, oracle.Params(**base), sigma=1e-3, seed=77, signal=0)
    r1 = oracle.multiphaseshift(w, a, oracle.Params(**base, tau_noise=3e-3), sigma=1e-3,
                                seed=77, signal=0)
    o = np.lexsort(w.T[::-1])
    assert r1.status == 0 and np.array_equal(r1.freqs, w[o])
    assert r1.trace[0]["n_acc"] > r0.trace[0]["n_acc"]


# ------------------------------------------------- R19: Philox word layout ----

def _box_muller(w_radial: int, w_angle: int, sigma: float) -> complex:
    """sigma / sqrt(2) sqrt(-2 ln(1 - u1)) e^{2 pi i u2}, u = top 53 bits * 2^-53."""
    u1 = (w_radial >> 11) * 2.0 ** -53
    u2 = (w_angle >> 11) * 2.0 ** -53
    r = math.sqrt(-2.0 * math.log1p(-u1))
    return sigma / math.sqrt(2.0) * r * complex(math.cos(2 * math.pi * u2),
                                                math.sin(2 * math.pi * u2))


def test_noise_words_from_known_answer_vector():
    """seed 0, signal 0, round 0, set 0: samples h = 0 and h = 1 share counter (0, 0, 0, 0),
    the Random123 known-answer block; h = 0 takes words 0 (radial) and 1 (angle), h = 1
    words 2 and 3."""
    out = [int(x, 16) for x in GOLD["philox4x64_10_kat"]["out"]]
    got = philox.sample_noise(0, 0, 0, 0, np.array([0, 1, 1, 0]), sigma=0.5)
    want0 = _box_muller(out[0], out[1], 0.5)
    want1 = _box_muller(out[2], out[3], 0.5)
    assert abs(got[0] - want0) < 1e-15 and abs(got[3] - want0) < 1e-15
    assert abs(got[1] - want1) < 1e-15 and abs(got[2] - want1) < 1e-15
    # the mix-ups this rules out
    assert abs(want0 - _box_muller(out[1], out[0], 0.5)) > 1e-3
    assert abs(want0 - want1) > 1e-3


def test_noise_counter_layout():
    """h = 2, 3 use counter (1, s, round, 0); the set and round enter words 1 and 2 of the
    counter and the signal the second key word (checked against philox4x64_10 directly)."""
    seed, sig, rnd, s = 12345, 6, 3, 2
    out = philox.philox4x64_10([np.uint64(1), np.uint64(s), np.uint64(rnd), np.uint64(0)],
                               [np.uint64(seed), np.uint64(sig)])
    out = [int(x) for x in out]
    got = philox.sample_noise(seed, sig, rnd, s, np.array([2, 3]), sigma=1.0)
    assert abs(got[0] - _box_muller(out[0], out[1], 1.0)) < 1e-15
    assert abs(got[1] - _box_muller(out[2], out[3], 1.0)) < 1e-15


# ------------------------------------------------ classifier feature axis n* ---

def _bucket(d2, K, NB, y, F0, dev_coarse, dev_fine):
    """Spectra of bucket 0 for a mode at unwrapped y: F_n = F_0 e^{i pi y_n / NB} (1 + dc_n),
    F_{d2+n} = F_0 e^{i pi K y_n / NB} (1 + df_n) (sets s = n and d2 + n, eq. (41))."""
    F = np.zeros((2 * d2 + 1, 3), dtype=np.complex128)
    F[0, 0] = F0
    for n in range(1, d2 + 1):
        F[n, 0] = F0 * np.exp(1j * math.pi * y[n - 1] / NB) * (1 + dev_coarse[n - 1])
        F[d2 + n, 0] = F0 * np.exp(1j * math.pi * K * y[n - 1] / NB) * (1 + dev_fine[n - 1])
    return F


def test_feature_axis_is_the_worst_fine_ratio():
    d2, K, NB, s = 4, 8, 1 << 12, 1e-3
    y = [5, -17, 300, 41]
    m = 2
    dc = [0.0, 2e-4 + 1e-4j, 3e-3, -5e-4j]
    # fine deviations: axis 3 has the largest coarse deviation but axis 4 the largest fine
    df = [0.0, -3e-4j, 1e-3, 4e-3]
    F = _bucket(d2, K, NB, y, 1.5 - 0.5j, dc, df)
    f = C.bucket_features(F, 0, y, m, d2, K, NB, s)
    want = []
    for dv in (dc[m - 1], df[m - 1], dc[3], df[3]):   # (m coarse, m fine, n* coarse, n* fine)
        want += [math.asinh(dv.real / s), math.asinh(dv.imag / s)]
    assert np.allclose(f, want, rtol=0, atol=1e-9)


def test_feature_axis_ties_go_to_the_smaller_axis():
    d2, K, NB, s = 3, 4, 1 << 10, 1e-3
    y = [7, 7, 7]              # equal phases: axes 2 and 3 get bit-identical spectra
    m = 1
    dc = [0.0, 1e-3, 2e-3]
    df = [0.0, 5e-3, 5e-3]
    F = _bucket(d2, K, NB, y, 2.0, dc, df)
    f = C.bucket_features(F, 0, y, m, d2, K, NB, s)
    assert abs(f[4] - math.asinh(1e-3 / s)) < 1e-9     # axis 2's coarse deviation, not 3's


def test_feature_axis_without_ladder_and_single_axis():
    # no ladder: "fine" is the coarse set, so n* is chosen by the coarse ratios
    d2, NB, s = 3, 1 << 10, 1e-3
    y = [3, -9, 11]
    F = np.zeros((d2 + 1, 1), dtype=np.complex128)
    F[0, 0] = 1.0
    dev = [0.0, 2e-3, -6e-3]
    for n in range(1, d2 + 1):
        F[n, 0] = np.exp(1j * math.pi * y[n - 1] / NB) * (1 + dev[n - 1])
    f = C.bucket_features(F, 0, y, 1, d2, 1, NB, s)
    assert abs(f[4] - math.asinh(-6e-3 / s)) < 1e-9 and abs(f[6] - f[4]) < 1e-12
    # d2 = 1: n* = m
    F1 = F[:2].copy()
    f1 = C.bucket_features(F1, 0, y[:1], 1, 1, 1, NB, s)
    assert np.allclose(f1[4:], f1[:4], rtol=0, atol=0)


# ------------------------------------------------------ decision margins -----

def test_test_margin_is_the_distance_to_the_threshold():
    # tau = 2^-10, deviations 2^-11 (set 1) and 3 * 2^-12 (set 2): distances 2^-11, 2^-12
    p, F0 = 64, 8.0
    F = _spectra_with_ratios(F0, [1.0 + 2 ** -11, 1.0 - 3 * 2 ** -12], p)
    P = oracle.Params(d=2, N=64, k=1, tau=2 ** -10)
    assert M._test_margin(F, 0, p, P) == 2 ** -12


def test_select_margin_counts_only_candidate_ties():
    absF0 = np.array([50.0, 40.0, 39.0, 0.001, 0.0005])
    order = np.argsort(-absF0, kind="stable")
    # cut between 40 and 39 (both candidates at p = 10, eta = 1e-3): gap 1 / p = 0.1
    assert abs(M._select_margin(absF0, order, 2, 10, 1e-3) - 0.1) < 1e-15
    # cut between two buckets below the floor: only the floor distances count
    # (0.001 / 10 = 1e-4 against eta = 1e-3: 9e-4)
    assert abs(M._select_margin(absF0, order, 4, 10, 1e-3) - 9e-4) < 1e-15


def test_noiseless_recovery_margins_are_wide():
    import workloads
    w, a = workloads.planted_signal(1000, 0, 2, 64, 8)
    r = oracle.multiphaseshift(w, a, oracle.Params(d=2, N=64, k=8, tau=1e-6))
    assert all(t["margin_coeff"] > 0.5e-3 and t["margin_ratio"] > 1e-7 for t in r.trace)
