"""Write the oracle's expected results for full-size signals of the large workloads.

This script calls only the FP64 CPU oracle (`oracle/`) and the seeded input
generators (`workloads/`); nothing here comes from the HIP path.  The oracle
takes minutes per signal at these sizes, too long to run inside a GPU test, so
its results are stored under tests/golden/ and the GPU tests compare the
library's launch with them.

    python tests/golden/make_goldens.py              # every case
    python tests/golden/make_goldens.py c5_full      # one case

Each signal becomes one compressed .npz file holding the recovered frequencies
(int64 [k_found, d], lexicographic order of w), coefficients (complex128), the
status, rounds and samples, the per-round trace rows (i, k*, p, m, candidates,
accepted, |R|, verification flag), each round's smallest decision margins (how near a
tie its ratio tests came, in units of the ratio, and its candidate cut, eta floor and
verification count, in units of |F|/p), and a digest of the planted input so that a
test can tell that it regenerated the same signal.  The recipe and method
parameters are stored beside them as JSON text.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time
from multiprocessing import get_context

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

# name: recipe, overrides, batch size, sparsity, signals stored.  The batch size
# is the launch the GPU test runs (signal b of a batch does not depend on B).
CASES = {
    # the large workload at its recipe: 64 signals, d = 20, N = 65536, k = 4096,
    # sigma = 1e-2, c = 1.99 (first prime 8161)
    "c5_full": dict(recipe="c5", over={}, B=64, k=4096, signals=(0, 1)),
    # the same batch at c = 1.49 (first prime 6143), a value the autotuner may pick
    "c5_full_c149": dict(recipe="c5", over={"c": 1.49}, B=64, k=4096, signals=(0, 1)),
    # and at c = 2.5 (first prime 10243: Bluestein length 32768, past the in-LDS FFT)
    "c5_full_c25": dict(recipe="c5", over={"c": 2.5}, B=64, k=4096, signals=(0, 1)),
    # and at c = 3 (first prime 12301: the sampler keeps half the twiddle table)
    "c5_full_c30": dict(recipe="c5", over={"c": 3.0}, B=64, k=4096, signals=(0, 1)),
    # the classifier workload's signals at full size, plain ratio test: d = 6, N = 4096,
    # k = 2000, sigma ~ U[0, 1e-2] per signal.  Signals 3 and 11 are the two least noisy of
    # the 16 (sigma 1.07e-3 and 1.31e-3): above sigma ~ 3e-3 the plain test's decisions
    # come within the FP32 spectra's rounding of their thresholds (the oracle's decision
    # margins drop to ~1e-3 of the threshold), so that the FP32 path and the FP64 oracle
    # may take different but equally valid paths
    "c4_full": dict(recipe="c4", over={}, B=16, k=2000, signals=(3, 11),
                    sigma_uniform=(0.0, 1e-2)),
}


def batch_for(case: dict):
    """The planted batch of a case (the GPU test draws the same one)."""
    cfg = workloads.config(case["recipe"], **case["over"])
    B = case["B"]
    if "sigma_uniform" in case:
        lo, hi = case["sigma_uniform"]
        sigma = workloads.planted.uniform_sigma(cfg["seed"], B, lo, hi)
    else:
        sigma = cfg["sigma"]
    pb = workloads.planted_batch(cfg["seed"], B, cfg["d"], cfg["N"], case["k"], cfg["mag"], sigma)
    return cfg, pb


def oracle_params(cfg: dict, k: int) -> oracle.Params:
    return oracle.Params(d=cfg["d"], N=cfg["N"], k=int(k), d1=cfg["d1"], c=cfg["c"],
                         ladder_K=cfg["ladder_K"], tau=cfg["tau"], eta=cfg["eta"],
                         p_min=cfg["p_min"], robust=cfg["robust"], verify=cfg["verify"],
                         verify_eta=cfg["verify_eta"], blocks=cfg["blocks"],
                         order=cfg["order"], tilt=cfg["tilt"],
                         max_rounds=cfg.get("max_rounds", 64))


def planted_digest(w: np.ndarray, a: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(w, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(a, dtype=np.complex128).tobytes())
    return h.hexdigest()


def golden_path(name: str, b: int) -> str:
    return os.path.join(HERE, f"{name}_s{b}.npz")


def _one(job):
    name, b = job
    case = CASES[name]
    cfg, pb = batch_for(case)
    w, a = pb.signal(b)
    t0 = time.time()
    r = oracle.multiphaseshift(w, a, oracle_params(cfg, pb.k[b]), sigma=float(pb.sigma[b]),
                               seed=pb.seed, signal=b)
    secs = time.time() - t0
    trace = np.array([[t["i"], t["kstar"], t["p"], t["m"], t["n_cand"], t["n_acc"], t["n_R"],
                       t["verify"]] for t in r.trace], dtype=np.int64).reshape(-1, 8)
    margin_ratio = np.array([t["margin_ratio"] for t in r.trace], dtype=np.float64)
    margin_coeff = np.array([t["margin_coeff"] for t in r.trace], dtype=np.float64)
    meta = dict(case=name, signal=b, recipe=case["recipe"], over=case["over"], B=case["B"],
                k=case["k"], sigma=float(pb.sigma[b]), seed=pb.seed, c=cfg["c"],
                oracle_seconds=round(secs, 1), planted_sha256=planted_digest(w, a),
                writer="tests/golden/make_goldens.py (FP64 oracle only)")
    np.savez_compressed(golden_path(name, b), freqs=r.freqs.astype(np.int64),
                        coeffs=r.coeffs.astype(np.complex128),
                        status=np.int64(r.status), rounds=np.int64(r.rounds),
                        samples=np.int64(r.samples), trace=trace, margin_ratio=margin_ratio,
                        margin_coeff=margin_coeff,
                        meta=np.array(json.dumps(meta, sort_keys=True)))
    return name, b, r.status, r.rounds, secs


def main(argv):
    names = argv or list(CASES)
    jobs = [(n, b) for n in names for b in CASES[n]["signals"]]
    procs = min(len(jobs), max(1, (os.cpu_count() or 2) - 1))
    with get_context("spawn").Pool(procs) as pool:
        for name, b, status, rounds, secs in pool.imap_unordered(_one, jobs):
            print(f"{name} signal {b}: status {status}, {rounds} rounds, {secs:.0f} s",
                  flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
