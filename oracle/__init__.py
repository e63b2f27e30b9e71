"""Plain FP64 CPU oracle for the MultiPhaseshift sparse Fourier method.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference the HIP
path is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does and
shares no code with it.

It follows the paper "High-Dimensional Sparse Fourier Algorithms" (Choi,
Christlieb, Wang): the 1-D Phaseshift algorithm of Section 2.1, the partial
unwrapping of Section 4.1.2 (eqs. (35)-(42)) and the MultiPhaseshift
procedure of the same section, explained in Section 5.0.  Every function
cites the passage it follows.  Points where the paper is silent or
inconsistent are resolved as listed in `READINGS` below.

Parity pins (tests under tests/test_oracle_*.py): closed forms of eqs. (3)
and (41), a brute-force O(p^2) DFT, exhaustive unwrap/wrap bijections, the
k = 1 special case, brute-force d-dimensional DFTs on tiny full grids (uniform
and uneven partitions, shuffled coordinate orders, a hand-computed unwrapping), exact
recovery of planted spectra, the d = 1 reduction to Phaseshift, per-round
isolation statistics, the Philox known-answer vector, the closed form of the
verification line (R14) and the false-accept experiment it is there for; the
learned classifier (classifier.py) is pinned by finite differences, a
hand-computed network and the feature definitions.
"""
from .primes import is_prime, ith_prime_at_least, primes_upto
from .unwrapping import partition, unwrap_matrix, unwrap, wrap, y_range
from .philox import philox4x64_10, sample_noise
from .signal import evaluate, sample_points
from .transforms import dft_direct, dft
from .phaseshift import phaseshift_1d
from .method import Params, Result, multiphaseshift, round_samples, shift_table, READINGS

__all__ = [
    "is_prime", "ith_prime_at_least", "primes_upto",
    "partition", "unwrap_matrix", "unwrap", "wrap", "y_range",
    "philox4x64_10", "sample_noise", "evaluate", "sample_points",
    "dft_direct", "dft", "phaseshift_1d",
    "Params", "Result", "multiphaseshift", "round_samples", "shift_table", "READINGS",
]
