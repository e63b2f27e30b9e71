"""Pins of the whole oracle: closed forms per round, special cases, brute force, truth."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from oracle import unwrapping as uw
from oracle import method as mps_mod
from oracle import signal as sig_mod

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _run(name, b=0, **over):
    cfg = workloads.config(name, **over)
    B = max(b + 1, 1)
    batch = workloads.planted_batch(cfg["seed"], B, cfg["d"], cfg["N"],
                                    cfg["k"] if not isinstance(cfg["k"], tuple) else 500,
                                    cfg["mag"], cfg["sigma"] if not isinstance(cfg["sigma"], tuple) else 0.0)
    w, a = batch.signal(b)
    P = oracle.Params(d=cfg["d"], N=cfg["N"], k=int(batch.k[b]), d1=cfg["d1"], c=cfg["c"],
                      ladder_K=cfg["ladder_K"], tau=cfg["tau"], eta=cfg["eta"],
                      p_min=cfg["p_min"], robust=cfg["robust"], blocks=cfg["blocks"],
                      order=cfg["order"])
    return w, a, P, batch


def _closed_form(y_pl, a_pl, y_R, a_R, P, p, m, tab):
    """eq. (41): F_s[h] = p sum_{y_m = h mod p} a e^{2 pi i eps K_s y_{n_s}} over planted minus R."""
    S = len(tab)
    F = np.zeros((S + 1, p), complex)
    for ys, as_, sign in ((y_pl, a_pl, 1.0), (y_R, a_R, -1.0)):
        for y, a in zip(ys, as_):
            hb = int(y[m - 1]) % p
            F[0, hb] += sign * p * a
            for s, (n, K) in enumerate(tab, start=1):
                F[s, hb] += sign * p * a * np.exp(2j * np.pi * P.eps * K * int(y[n - 1]))
    return F


@pytest.mark.parametrize("name,over", [("c1", {}), ("c1", {"d1": 2}), ("c2", {}),
                                       ("e4", {}), ("c3b", {"k": 60, "sigma": 0.0}),
                                       ("e1", {"k": 24}), ("e2", {"k": 12}), ("e3", {}),
                                       ("c2", {"blocks": (2, 1, 1), "order_seed": 2001})])
def test_round_spectra_match_eq41(name, over):
    w, a, P, _ = _run(name, **over)
    r = oracle.multiphaseshift(w, a, P, keep_spectra=True)
    y_pl = uw.unwrap(w, P.d1, P.N, P.blocks, P.order)
    tab = oracle.shift_table(P.d2, P.ladder_K)
    for tr, F, (yR, aR) in zip(r.trace, r.spectra, r.registry):
        ref = _closed_form(y_pl, a, yR, aR, P, tr["p"], tr["m"], tab)
        scale = tr["p"] * np.abs(a).max()
        tol = 1e-12 if P.NB < 1e5 else 1e-9
        assert np.abs(F - ref).max() <= tol * scale * max(1, len(a))


@pytest.mark.parametrize("d,N,d1", [(1, 64, 1), (2, 64, 1), (2, 64, 2), (5, 1024, 1),
                                    (20, 20, 4), (12, 20, 3)])
def test_single_mode_round_one(d, N, d1):
    # k = 1: one bucket, ratios e^{2 pi i eps y_n}, decode exact in round 1 (eq. (4)-(7))
    rng = np.random.default_rng(d * 1000 + N)
    for _ in range(5):
        w = rng.integers(-N // 2, N // 2, size=(1, d))
        a = np.exp(2j * np.pi * rng.uniform(size=1)) * rng.uniform(1, 3)
        r = oracle.multiphaseshift(w, a, oracle.Params(d=d, N=N, k=1, d1=d1))
        assert r.rounds == 1 and r.status == 0
        assert np.array_equal(r.freqs, w)
        assert abs(r.coeffs[0] - a[0]) < 1e-9


@pytest.mark.parametrize("d,N,blocks", [(7, 20, (4, 3)), (5, 64, (2, 1, 2)), (3, 1024, (1, 2))])
def test_single_mode_round_one_uneven(d, N, blocks):
    # k = 1 with blocks of different sizes (d prime: Section 4.1.2) over a random order:
    # the ratios are e^{2 pi i eps y_n} with one eps = 1/(2 N^max d_q), exact in round 1
    rng = np.random.default_rng(d * 7 + N)
    for _ in range(5):
        order = tuple(int(x) for x in rng.permutation(d))
        w = rng.integers(-N // 2, N // 2, size=(1, d))
        a = np.exp(2j * np.pi * rng.uniform(size=1)) * rng.uniform(1, 3)
        P = oracle.Params(d=d, N=N, k=1, blocks=blocks, order=order)
        assert P.NB == N ** max(blocks)
        r = oracle.multiphaseshift(w, a, P)
        assert r.rounds == 1 and r.status == 0
        assert np.array_equal(r.freqs, w)
        assert abs(r.coeffs[0] - a[0]) < 1e-9


def _bruteforce_spectrum(w, a, d, N):
    # f on the full grid (Z_N / N)^d, then the d-dim DFT / N^d (Section 2.2's setting)
    grid = np.stack(np.meshgrid(*[np.arange(N) / N] * d, indexing="ij"), axis=-1).reshape(-1, d)
    f = oracle.evaluate(w, a, grid).reshape([N] * d)
    A = np.fft.fftn(f) / N ** d
    idx = np.argwhere(np.abs(A) > 1e-8)
    freqs = np.where(idx >= N // 2, idx - N, idx).astype(np.int64)
    coeffs = A[tuple(idx.T)]
    order = np.lexsort(freqs.T[::-1])
    return freqs[order], coeffs[order]


@pytest.mark.parametrize("d,N,d1,k,seed", [(2, 64, 1, 8, 1000), (2, 64, 2, 8, 1001),
                                           (3, 16, 1, 6, 7), (4, 8, 2, 5, 9),
                                           (6, 4, 3, 4, 11)])
def test_bruteforce_full_grid(d, N, d1, k, seed):
    w, a = workloads.planted_signal(seed, 0, d, N, k)
    fw, fa = _bruteforce_spectrum(w, a, d, N)
    assert fw.shape == (k, d)
    r = oracle.multiphaseshift(w, a, oracle.Params(d=d, N=N, k=k, d1=d1))
    assert r.status == 0
    assert np.array_equal(r.freqs, fw)
    assert np.abs(r.coeffs - fa).max() < 1e-9


@pytest.mark.parametrize("d,N,blocks,order,k,seed", [(3, 16, (2, 1), (2, 0, 1), 6, 21),
                                                     (5, 4, (3, 2), (3, 1, 4, 0, 2), 5, 23),
                                                     (4, 8, (1, 3), (3, 2, 1, 0), 5, 25)])
def test_bruteforce_full_grid_uneven(d, N, blocks, order, k, seed):
    # general partitions recover what the d-dim DFT of the full grid finds
    w, a = workloads.planted_signal(seed, 0, d, N, k)
    fw, fa = _bruteforce_spectrum(w, a, d, N)
    assert fw.shape == (k, d)
    r = oracle.multiphaseshift(w, a, oracle.Params(d=d, N=N, k=k, blocks=blocks, order=order))
    assert r.status == 0
    assert np.array_equal(r.freqs, fw)
    assert np.abs(r.coeffs - fa).max() < 1e-9


@pytest.mark.parametrize("N,k,seed", [(16, 6, 31), (8, 5, 33)])
def test_bruteforce_full_grid_tilted(N, k, seed):
    # the tilted recovery (R23) finds what the 2-dim DFT of the full grid finds
    w, a = workloads.planted_signal(seed, 0, 2, N, k)
    fw, fa = _bruteforce_spectrum(w, a, 2, N)
    r = oracle.multiphaseshift(w, a, oracle.Params(d=2, N=N, k=k, tilt=True))
    assert r.status == 0
    assert np.array_equal(r.freqs, fw)
    assert np.abs(r.coeffs - fa).max() < 1e-9


@pytest.mark.parametrize("N,r", [(64, 4), (64, 6), (1024, 5)])
def test_worst_case_rectangles_need_tilting(N, r):
    # Section 3.3: frequencies on the vertices of axis-aligned rectangles collide on every
    # parallel projection, so the untilted method recovers nothing; tilted with the
    # triple of Theorem 1 it recovers all of them
    pb = workloads.rectangle_batch(7000 + N + r, 3, N, r)
    for b in range(pb.B):
        w, a = pb.signal(b)
        o = np.lexsort(w.T[::-1])
        plain = oracle.multiphaseshift(w, a, oracle.Params(d=2, N=N, k=r * r, max_rounds=8))
        assert plain.status == 1 and plain.freqs.shape[0] == 0
        P = oracle.Params(d=2, N=N, k=r * r, tilt=True)
        res = oracle.multiphaseshift(w, a, P)
        assert res.status == 0
        assert np.array_equal(res.freqs, w[o])
        assert np.abs(res.coeffs - a[o]).max() < 1e-9


# coefficient tolerance: 1e-9, and 1e-8 for the d = 100 and 1000 recipes, where the oracle
# evaluates exp(2 pi i w . t) at arguments of up to N^d1 / 2 = 1.6e6 cycles in FP64
# (a phase error of about 1e-9 rad per term)
@pytest.mark.parametrize("name,over,trials,tol", [("c1", {}, 40, 1e-9), ("c1", {"d1": 2}, 20, 1e-9),
                                                  ("c2", {}, 3, 1e-9), ("e4", {}, 3, 1e-9),
                                                  ("e1", {"k": 32}, 3, 1e-8),
                                                  ("e2", {"k": 16}, 2, 1e-8),
                                                  ("e3", {}, 3, 1e-9),
                                                  ("c2", {"blocks": (2, 1, 1),
                                                          "order_seed": 2001}, 2, 1e-9)])
def test_exact_recovery_noiseless(name, over, trials, tol):
    cfg = workloads.config(name, **over)
    for t in range(trials):
        w, a = workloads.planted_signal(cfg["seed"] + t, 0, cfg["d"], cfg["N"], cfg["k"], cfg["mag"])
        P = oracle.Params(d=cfg["d"], N=cfg["N"], k=cfg["k"], d1=cfg["d1"], c=cfg["c"],
                          tau=cfg["tau"], eta=cfg["eta"], blocks=cfg["blocks"],
                          order=cfg["order"])
        r = oracle.multiphaseshift(w, a, P)
        o = np.lexsort(w.T[::-1])
        assert r.status == 0
        assert np.array_equal(r.freqs, w[o])
        assert np.abs(r.coeffs - a[o]).max() < tol


def test_noisy_recovery_c3_small():
    # noise ladder: support exact, coefficient error of order sigma / sqrt(p)
    cfg = workloads.config("c3b")
    batch = workloads.planted_batch(cfg["seed"], 1, cfg["d"], cfg["N"], 120, cfg["mag"], cfg["sigma"])
    w, a = batch.signal(0)
    P = oracle.Params(d=10, N=65536, k=120, c=3.0, ladder_K=1024, tau=1e-3, eta=1e-3,
                      p_min=101, robust=True)
    r = oracle.multiphaseshift(w, a, P, sigma=1e-3, seed=batch.seed, signal=0)
    o = np.lexsort(w.T[::-1])
    assert np.array_equal(r.freqs, w[o])
    assert np.abs(r.coeffs - a[o]).max() < 20 * 1e-3 / math.sqrt(101)


def test_one_dim_reduces_to_phaseshift():
    # d = d1 = d2 = 1: MultiPhaseshift is the Phaseshift algorithm of Section 2.1
    for seed in range(5):
        w, a = workloads.planted_signal(70 + seed, 0, 1, 4096, 40, (1.0, 2.0))
        r = oracle.multiphaseshift(w, a, oracle.Params(d=1, N=4096, k=40))
        w1, a1, tr1 = oracle.phaseshift_1d(w[:, 0], a, k=40, N=4096)
        assert [t["p"] for t in r.trace] == [t["p"] for t in tr1]
        assert [t["n_acc"] for t in r.trace] == [t["n_acc"] for t in tr1]
        assert np.array_equal(r.freqs[:, 0], w1)
        assert np.allclose(r.coeffs, a1, atol=1e-12)
        assert np.array_equal(np.sort(w[:, 0]), w1)


def test_isolation_fraction_round_one():
    # c = 5, N >= 5k: at least 80% of modes isolated mod p and by projection (Analysis section)
    frac = []
    for seed in range(8):
        w, a = workloads.planted_signal(500 + seed, 0, 4, 8192, 200, (1.0, 2.0))
        r = oracle.multiphaseshift(w, a, oracle.Params(d=4, N=8192, k=200, c=5.0))
        frac.append(r.trace[0]["n_acc"] / 200)
    assert np.mean(frac) >= GOLD["isolation"]["isolated_mod_p_and_N"]


def test_sample_count_grows_with_d():
    # samples per round are (d2 + 1) p: linear in d at fixed k (Theta(dk), Section 5.2)
    s = []
    for d in (2, 4, 8):
        w, a = workloads.planted_signal(900, 0, d, 4096, 64, (1.0, 2.0))
        r = oracle.multiphaseshift(w, a, oracle.Params(d=d, N=4096, k=64, c=5.0))
        assert r.status == 0
        s.append(r.samples / (d + 1))
    assert max(s) / min(s) < 2.0


def test_not_converged_status():
    w, a = workloads.planted_signal(1, 0, 2, 64, 8)
    r = oracle.multiphaseshift(w, a, oracle.Params(d=2, N=64, k=8, max_rounds=1))
    assert r.rounds == 1 and r.status == 1 and r.freqs.shape[0] < 8


# ---- planted mistakes: each must be caught by one of the pins above -----------------------

def _pins_hold(monkeypatch=None):
    try:
        test_round_spectra_match_eq41("c1", {})
        test_exact_recovery_noiseless("c1", {}, 5, 1e-9)
        test_single_mode_round_one(2, 64, 1)
        test_bruteforce_full_grid(2, 64, 2, 8, 1001)
        test_bruteforce_full_grid_uneven(3, 16, (2, 1), (2, 0, 1), 6, 21)
        test_bruteforce_full_grid_tilted(16, 6, 31)
    except AssertionError:
        return False
    return True


def test_pins_hold_unmutated():
    assert _pins_hold()


@pytest.mark.parametrize("mutation", ["dft_sign", "unwrap_power", "no_residual",
                                      "shift_axis", "coef_scale", "arg_sign", "round_floor",
                                      "wrap_natural_order", "block_digits_reversed",
                                      "tilt_back_transposed", "tilt_sample_unrotated"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "dft_sign":
        monkeypatch.setattr(mps_mod, "dft", lambda v: np.fft.ifft(v) * v.shape[-1])
    elif mutation == "unwrap_power":
        orig = sig_mod.unwrap_matrix
        monkeypatch.setattr(sig_mod, "unwrap_matrix",
                            lambda d, d1, N, *part: orig(d, d1, N, *part) * N)
    elif mutation == "no_residual":
        monkeypatch.setattr(mps_mod, "_residual", lambda yR, aR, p, m, n, shift: np.zeros(p, complex))
    elif mutation == "shift_axis":
        orig = sig_mod.sample_points
        monkeypatch.setattr(mps_mod, "sample_points",
                            lambda d, d1, N, p, m, n, shift, *part:
                            orig(d, d1, N, p, m, m, shift, *part))
    elif mutation == "coef_scale":
        monkeypatch.setattr(mps_mod, "_coefficient", lambda F0h, p: complex(F0h) / (p - 1))
    elif mutation == "arg_sign":
        monkeypatch.setattr(mps_mod, "_arg", lambda z: -math.atan2(z.imag, z.real))
    elif mutation == "round_floor":
        # R11 misread: truncation towards -inf instead of rounding to nearest
        monkeypatch.setattr(mps_mod, "_round_half_away", lambda x: math.floor(x))
    elif mutation == "wrap_natural_order":
        # R22 misread: the answer wrapped back without the coordinate order
        orig = uw.wrap
        monkeypatch.setattr(mps_mod, "wrap",
                            lambda y, d1, N, blocks=None, order=None: orig(y, d1, N, blocks))
    elif mutation == "block_digits_reversed":
        # R22 misread: the last coordinate of a block is the least significant digit
        orig = sig_mod.unwrap_matrix

        def rev(d, d1, N, blocks=None, order=None, tilt=None):
            b, o, s = uw.partition(d, d1, blocks, order)
            o2 = sum((tuple(reversed(o[s[q]:s[q + 1]])) for q in range(len(b))), ())
            return orig(d, d1, N, blocks, o2, tilt)
        monkeypatch.setattr(sig_mod, "unwrap_matrix", rev)
    elif mutation == "tilt_back_transposed":
        # R23 misread: rotated back with U^T instead of U
        monkeypatch.setattr(mps_mod, "tilt_back",
                            lambda y, a, b, c, N: uw.tilt_back(y, -a, b, c, N))
    elif mutation == "tilt_sample_unrotated":
        # R23 misread: the samples taken on the unrotated axes
        orig = sig_mod.unwrap_matrix
        monkeypatch.setattr(sig_mod, "unwrap_matrix",
                            lambda d, d1, N, blocks=None, order=None, tilt=None:
                            orig(d, d1, N, blocks, order, None))
    assert not _pins_hold()


def test_round_samples_point_subset():
    """Sampling only some points h gives exactly those columns of the full sets."""
    w, a = workloads.planted_signal(31, 0, 3, 256, 20, (1.0, 2.0))
    P = oracle.Params(d=3, N=256, k=20, ladder_K=8)
    yR = oracle.unwrap(w[:3], 1, 256)
    aR = a[:3] * 0.5
    full = oracle.round_samples(w, a, P, 61, 2, 2, yR, aR, sigma=0.1, seed=5, signal=1)
    hs = np.array([60, 0, 17, 17, 33])
    part = oracle.round_samples(w, a, P, 61, 2, 2, yR, aR, sigma=0.1, seed=5, signal=1, hs=hs)
    assert np.array_equal(part, full[:, hs])


def test_verification_line_closed_form():
    """R14 samples: their DFT is p times the residual's bucket sums, bucket of a
    mode = (y . v) mod p with v_n = q^(n-1) mod p (eq. (3) on the tilted line)."""
    w, a = workloads.planted_signal(41, 0, 4, 64, 40, (1.0, 2.0))
    P = oracle.Params(d=4, N=64, k=40, d1=2)
    y = oracle.unwrap(w, 2, 64)
    yR = np.vstack([y[:5], y[:1] + np.array([1, 0])])      # 5 exact entries + 1 wrong one
    aR = np.concatenate([a[:5] * 0.75, [0.3 + 0.1j]])
    p, q = 101, 7
    F = np.fft.fft(oracle.method.verify_samples(w, a, P, p, q, 3, yR, aR))
    v = np.array([1, q], dtype=np.int64)
    want = np.zeros(p, complex)
    np.add.at(want, (y @ v) % p, a)
    np.add.at(want, (yR @ v) % p, -aR)
    assert np.abs(F / p - want).max() < 1e-9


def test_verification_catches_false_accepts():
    """R14 catching classifier errors: with the ratio test switched off (tau = 10 accepts every
    in-band decode) and c = 1.5, the plain loop ends at |R| = k with wrong entries
    and status OK; with verification every OK result is the planted spectrum."""
    silent_wrong = exact_verified = 0
    for seed in range(8):
        w, a = workloads.planted_signal(800 + seed, 0, 3, 64, 30, (1.0, 2.0))
        o = np.lexsort(w.T[::-1])
        for verify in (False, True):
            P = oracle.Params(d=3, N=64, k=30, c=1.5, tau=10.0, verify=verify,
                              verify_eta=1e-2)
            r = oracle.multiphaseshift(w, a, P)
            exact = r.freqs.shape == w.shape and np.array_equal(r.freqs, w[o])
            if verify:
                assert exact or r.status != oracle.method.STATUS_OK, seed
                exact_verified += int(exact)
                if exact:   # the run ends with one clean verification row
                    assert r.trace[-1]["verify"] == 1 and r.trace[-1]["n_cand"] == 0
            else:
                silent_wrong += int(r.status == oracle.method.STATUS_OK and not exact)
    assert silent_wrong >= 4 and exact_verified >= 6
