"""The library's kernels and host code run on the CPU in a host emulation (tests/emu):
a work-group is 256 host threads, __syncthreads() is a barrier that checks every
thread reaches the same one, the dynamic LDS is a heap block of exactly the launch's
size, and the FP32 matrix instruction exchanges its operands across the 64 threads of
its wave.  The same sources as the GPU build run under

  * AddressSanitizer + UndefinedBehaviorSanitizer: any access outside an allocation
    (LDS, workspace slots, inputs, outputs), undefined integer behaviour;
  * ThreadSanitizer: any two accesses to shared memory (LDS, __shared__ state,
    workspace) by different threads of a work-group that no barrier orders.

Each recovery is compared with the FP64 oracle as on the GPU: supports bit-exact,
statuses and per-round traces equal, coefficients within the path's tolerance.  The
deliberate defects of tests/emu/planted.cpp show that each check fires.
"""
import os
import shutil
import sys

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _emu():
    import emu
    return emu


def _params(sfft, cfg, k_max):
    return sfft.Params(d=cfg["d"], N=cfg["N"], k_max=k_max, d1=cfg["d1"], c=cfg["c"],
                       p_min=cfg["p_min"], ladder_K=cfg["ladder_K"], tau=(cfg["tau"] or 0.0),
                       eta=cfg["eta"], max_rounds=cfg.get("max_rounds", 64),
                       precision=sfft.SFFT_FP32 if cfg["precision"] == "fp32" else sfft.SFFT_FP64,
                       robust=int(cfg["robust"]), verify=int(cfg["verify"]),
                       verify_eta=cfg["verify_eta"] or 0.0, residual=int(cfg["residual"]),
                       blocks=cfg["blocks"], order=cfg["order"], tilt=1 if cfg["tilt"] else 0,
                       tilt_abc=(tuple(cfg["tilt"]) if isinstance(cfg["tilt"], tuple)
                                 else (0, 0, 0)))


def _oracle_params(cfg, k):
    return oracle.Params(d=cfg["d"], N=cfg["N"], k=int(k), d1=cfg["d1"], c=cfg["c"],
                         ladder_K=cfg["ladder_K"], tau=cfg["tau"], eta=cfg["eta"],
                         p_min=cfg["p_min"], robust=cfg["robust"], verify=cfg["verify"],
                         verify_eta=cfg["verify_eta"], blocks=cfg["blocks"],
                         order=cfg["order"], tilt=cfg["tilt"],
                         max_rounds=cfg.get("max_rounds", 64))


CASES = [
    # name, sanitizer, recipe, overrides, B, k, coefficient tolerance, entry point
    ("c1_fp64", "asan", "c1", {}, 2, 8, 1e-9, 0),
    ("c1_fp64", "tsan", "c1", {}, 2, 8, 1e-9, 0),
    ("c3_fp32_noisy", "asan", "c3b", {}, 2, 60, 1e-5, 0),
    ("c3_fp32_noisy", "tsan", "c3b", {}, 2, 60, 1e-5, 0),
    ("c3_fp32_residual_samples", "asan", "c3b", {"residual": 1}, 2, 60, 1e-5, 0),
    ("c3_fp32_static_scratch", "asan", "c3b", {}, 2, 60, 1e-5, 1),
    ("c3_fp32_static_scratch", "tsan", "c3b", {}, 2, 60, 1e-5, 1),
    ("c2_fp32", "asan", "c2", {}, 1, 64, 1e-5, 0),
    ("c1_fp64_tilt", "asan", "c1", {"tilt": True}, 2, 8, 1e-9, 0),
    ("e3_fp64_partition", "asan", "e3", {}, 1, 30, 1e-9, 0),
    # primes above the in-LDS DFT length: Bluestein lengths 16384 (FP64) and 32768 (FP32)
    # run as two halves through the workspace
    ("c1_fp64_long_dft", "asan", "c1", {"p_min": 4200}, 1, 8, 1e-9, 0),
    ("c1_fp64_long_dft", "tsan", "c1", {"p_min": 4200}, 1, 8, 1e-9, 0),
    ("c3_fp32_long_dft", "asan", "c3b", {"p_min": 8300}, 1, 20, 1e-5, 0),
    # verification lines of more than 1024 points: five consecutive points per thread
    ("c3_fp32_long_verify", "asan", "c3b", {"p_min": 1100}, 1, 20, 1e-5, 0),
    # several work-groups per signal: three launches per round, the sampling of each
    # line dealt out over 3 (FP32) or 2 (FP64) work-groups
    # (max_rounds bounds the launches: one pair per possible round)
    ("c3_fp32_split", "asan", "c3b", {"split": 3, "max_rounds": 12}, 2, 60, 1e-5, 0),
    ("c3_fp32_split", "tsan", "c3b", {"split": 3, "max_rounds": 12}, 2, 60, 1e-5, 0),
    ("c1_fp64_split", "asan", "c1", {"split": 2, "verify": True, "max_rounds": 8}, 2, 8,
     1e-9, 0),
    # verification lines of 1100+ points summed by the sampling launch's groups
    ("c3_fp32_split_long_verify", "asan", "c3b", {"p_min": 1100, "split": 3, "max_rounds": 12},
     1, 20, 1e-5, 0),
    ("c3_fp32_split_long_verify", "tsan", "c3b", {"p_min": 1100, "split": 3, "max_rounds": 12},
     1, 20, 1e-5, 0),
    # FP64 rounds whose DFTs (21 sets of 16384 points, in four parts) get a launch of
    # their own, dealt out over the groups
    ("e1_fp64_split_dft", "asan", "e1", {"p_min": 4200, "split": 2, "verify": False,
                                         "max_rounds": 2}, 1, 8, 1e-9, 0),
    # lines too long for the whole twiddle table next to six row tiles of staged A
    # fragments: the sampler keeps p/2 + 1 twiddles (and the recovery runs split)
    ("c5_fp32_half_table", "asan", "c5", {"p_min": 14500, "verify": False, "max_rounds": 2},
     1, 12, 1e-5, 0),
]


@pytest.mark.parametrize("name,kind,recipe,over,B,k,tol,entry", CASES,
                         ids=[f"{c[0]}-{c[1]}" for c in CASES])
def test_emulated_recovery_matches_oracle(name, kind, recipe, over, B, k, tol, entry):
    from paper_1606_07407_amd import sfft
    emu = _emu()
    over = dict(over)
    split = over.pop("split", 0)
    cfg = workloads.config(recipe, **over)
    pb = workloads.planted_batch(cfg["seed"], B, cfg["d"], cfg["N"], k, cfg["mag"], cfg["sigma"])
    prm = _params(sfft, cfg, k)
    prm.split_groups = split
    out = emu.run(kind, prm, pb, entry=entry)
    assert out["plan_status"] == 0 and out["call_status"] == 0, out["stderr"][-2000:]
    for b in range(B):
        w, a = pb.signal(b)
        ref = oracle.multiphaseshift(w, a, _oracle_params(cfg, k), sigma=float(pb.sigma[b]),
                                     seed=pb.seed, signal=b)
        kf = int(out["k_found"][b])
        assert int(out["status"][b]) == ref.status
        assert kf == ref.freqs.shape[0]
        assert np.array_equal(out["freqs"][b, :kf], ref.freqs)
        assert int(out["rounds"][b]) == ref.rounds and int(out["samples"][b]) == ref.samples
        want = np.array([[t["i"], t["kstar"], t["p"], t["m"], t["n_cand"], t["n_acc"],
                          t["n_R"], t["verify"]] for t in ref.trace])
        assert np.array_equal(out["trace"][b, :ref.rounds], want)
        if kf:
            rel = (np.abs(out["coeffs"][b, :kf] - ref.coeffs) / np.abs(ref.coeffs)).max()
            assert rel <= tol, rel


@pytest.mark.parametrize("kind,mode,expect", [
    ("tsan", "race", "ThreadSanitizer: data race"),
    ("asan", "oob", "heap-buffer-overflow"),
    ("asan", "diverge", "barrier divergence"),
    ("asan", "stall", "never completed"),
])
def test_emulator_checks_fire_on_planted_defects(kind, mode, expect):
    rc, err = _emu().run_planted(kind, mode)
    assert rc != 0 and expect in err, err[-2000:]


def test_emulator_clean_kernel_passes():
    rc, err = _emu().run_planted("tsan", "clean")
    assert rc == 0, err[-2000:]


@pytest.mark.parametrize("prec,p", [("fp64", 4093), ("fp64", 4099), ("fp64", 8191),
                                    ("fp32", 8191), ("fp32", 8209), ("fp32", 16381),
                                    ("fp32", 127), ("fp64", 127)])
def test_emulated_dft_matches_numpy(prec, p):
    """sfft_dft under ASan: short lengths transformed several sequences per pass, the
    longest in-LDS Bluestein lengths (8192 FP32, 4096 FP64) and the longer ones that run in
    two or four parts through the workspace."""
    from paper_1606_07407_amd import sfft
    emu = _emu()
    k_max = 3200 if prec == "fp32" else 1600
    params = sfft.Params(d=2, N=64, k_max=k_max, c=5.0,
                         precision=sfft.SFFT_FP32 if prec == "fp32" else sfft.SFFT_FP64)
    pb = workloads.planted_batch(1, 1, 2, 64, 1, (1.0, 2.0), 0.0)
    rng = np.random.default_rng(p)
    x = rng.normal(size=(5, p)) + 1j * rng.normal(size=(5, p))
    if prec == "fp32":
        x = x.astype(np.complex64).astype(np.complex128)
    out = emu.run("asan", params, pb, entry=2, dft_x=x)
    assert out["plan_status"] == 0 and out["call_status"] == 0, out["stderr"][-2000:]
    ref = np.fft.fft(x, axis=-1)
    L = 1 << int(np.ceil(np.log2(2 * p - 1)))
    u = 2.0 ** -24 if prec == "fp32" else 2.0 ** -53
    norm = np.sqrt((np.abs(x) ** 2).sum(axis=-1)).max()
    err = np.abs(out["dft"] - ref).max()
    assert err <= 8 * u * np.log2(L) * norm, err
