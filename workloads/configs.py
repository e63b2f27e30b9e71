"""Named workload recipes.

Each entry describes the synthetic signals (shape, sizes, value
distributions, noise) and the method parameters the measurements use for it.
The sizes follow the paper's own experiment (Section 5: d in {100, 1000},
d1 = 5, N = 20, c = 5, unit-magnitude random-phase coefficients) and the
measured single-GPU configurations:

  c1      d=2,  N=64,    k=8,    |a|=1,       noiseless, FP64, one signal
  c2      d=4,  N=1024,  k=256,  |a|~U[1,2],  noiseless, FP32 bulk, one signal
  c3a     d=10, N=65536, k~U{64..1024}, |a|~U[1,2], sigma=1e-3, B=512
  c3b     d=10, N=65536, k=1000, |a|~U[1,2], sigma=1e-3, B=512   (headline)
  c4      d=6,  N=4096,  k=2000, |a|~U[1,2], sigma~U[0,1e-2]  (classifier data)
  c5      d=20, N=65536, k=4096, |a|~U[1,4], sigma=1e-2, B=64  (p ~ 2k)
  e4      d=20, N=20, d1=4, k=100 (the worked example of Section 4.1)
  e1      d=100, N=20, d1=5, k in 2^0..2^9, |a|=1, noiseless, FP64, 100 trials
          (the paper's experiment at d = 100; k = 2^10 needs p > 4096, beyond
          the FP64 in-LDS DFT)
  e2      as e1 at d=1000 (d2 = 200 unwrapped coordinates, 201 sets per round)
  e3      e4 split unevenly as in Section 4.1: four blocks of 3 and two of 4, over a
          shuffled coordinate order

blocks / order_seed describe a general partition: block sizes (sum d; None:
uniform blocks of d1) and the seed of a random coordinate order (None: the
natural order), drawn here as a permutation of 0..d-1.  tilt (d = 2): True for
the rotated lines of Section 3.3 with the plan's triple, or a triple (a, b, c).
"""
from __future__ import annotations

import copy

import numpy as np

CONFIGS = {
    "c1": dict(d=2, N=64, k=8, B=1, mag=(1.0, 1.0), sigma=0.0, seed=1000,
               d1=1, c=5.0, ladder_K=1, tau=1e-6, eta=1e-3, precision="fp64",
               p_min=0, robust=False),
    "c2": dict(d=4, N=1024, k=256, B=1, mag=(1.0, 2.0), sigma=0.0, seed=2000,
               d1=1, c=5.0, ladder_K=1, tau=None, eta=1e-3, precision="fp32",
               p_min=0, robust=False),
    "c3a": dict(d=10, N=65536, k=(64, 1024), B=512, mag=(1.0, 2.0), sigma=1e-3,
                seed=3000, d1=1, c=3.0, ladder_K=1024, tau=1e-3, eta=1e-3,
                precision="fp32", p_min=101, robust=True, verify=True,
                verify_eta=1e-2),
    "c3b": dict(d=10, N=65536, k=1000, B=512, mag=(1.0, 2.0), sigma=1e-3,
                seed=3100, d1=1, c=3.0, ladder_K=1024, tau=1e-3, eta=1e-3,
                precision="fp32", p_min=101, robust=True, verify=True,
                verify_eta=1e-2),
    "c4": dict(d=6, N=4096, k=2000, B=512, mag=(1.0, 2.0), sigma=(0.0, 1e-2),
               seed=4000, d1=1, c=2.0, ladder_K=64, tau=1e-3, eta=1e-3,
               precision="fp32", p_min=101, robust=True, verify=True,
                verify_eta=1e-2),
    # c = 1.99: the first prime (8161) keeps the Bluestein length 2p - 1 within
    # the 16384-point in-LDS FFT
    "c5": dict(d=20, N=65536, k=4096, B=64, mag=(1.0, 4.0), sigma=1e-2,
               seed=5000, d1=1, c=1.99, ladder_K=256, tau=3e-3, eta=1e-3,
               precision="fp32", p_min=1009, robust=True, verify=True,
               verify_eta=1e-2),
    "e4": dict(d=20, N=20, k=100, B=1, mag=(1.0, 1.0), sigma=0.0, seed=6000,
               d1=4, c=5.0, ladder_K=1, tau=1e-6, eta=1e-8, precision="fp64",
               p_min=0, robust=False),
    "e1": dict(d=100, N=20, k=64, B=100, mag=(1.0, 1.0), sigma=0.0, seed=6100,
               d1=5, c=5.0, ladder_K=1, tau=1e-6, eta=1e-8, precision="fp64",
               p_min=0, robust=False),
    "e2": dict(d=1000, N=20, k=64, B=100, mag=(1.0, 1.0), sigma=0.0, seed=6200,
               d1=5, c=5.0, ladder_K=1, tau=1e-6, eta=1e-8, precision="fp64",
               p_min=0, robust=False),
    "e3": dict(d=20, N=20, k=100, B=1, mag=(1.0, 1.0), sigma=0.0, seed=6300,
               d1=4, blocks=(3, 3, 3, 3, 4, 4), order_seed=6301, c=5.0, ladder_K=1,
               tau=1e-6, eta=1e-8, precision="fp64", p_min=0, robust=False),
}


def config(name: str, **over):
    """A copy of the named recipe with fields overridden by keyword."""
    cfg = dict(verify=False, verify_eta=None, residual=0, blocks=None, order_seed=None,
               tilt=None)
    cfg.update(copy.deepcopy(CONFIGS[name]))
    cfg.update(over)
    cfg["name"] = name
    cfg["order"] = coordinate_order(cfg["order_seed"], cfg["d"])
    return cfg


def coordinate_order(seed, d: int):
    """A seeded random permutation of the d coordinates (None: natural order)."""
    if seed is None:
        return None
    return tuple(int(x) for x in np.random.default_rng(seed).permutation(d))
