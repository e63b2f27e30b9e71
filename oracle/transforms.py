"""The DFT of Section 2.1: F(b)[h] = sum_{j<M} b[j] exp(-2 pi i h j / M), unnormalised."""
from __future__ import annotations

import numpy as np


def dft_direct(b: np.ndarray) -> np.ndarray:
    """O(M^2) evaluation of the definition, with exact integer reduction of h j mod M."""
    b = np.asarray(b, dtype=np.complex128)
    M = b.shape[-1]
    hj = np.mod(np.outer(np.arange(M), np.arange(M)), M)
    W = np.exp(-2j * np.pi * hj / M)
    return b @ W.T


def dft(b: np.ndarray) -> np.ndarray:
    """The same transform via numpy's FFT (same sign and no normalisation)."""
    return np.fft.fft(np.asarray(b, dtype=np.complex128), axis=-1)
