"""Seeded synthetic planted-spectrum workloads.

This module only draws random inputs (integer frequency vectors and complex
coefficients) with the shapes and value distributions of the paper's
experiments and of the measured configurations.  It holds none of the sparse
Fourier method's arithmetic, so both the CPU oracle and the HIP path may take
their inputs from it.
"""
from .planted import PlantedBatch, planted_batch, planted_signal, rectangle_batch
from .configs import CONFIGS, config

__all__ = ["PlantedBatch", "planted_batch", "planted_signal", "rectangle_batch", "CONFIGS",
           "config"]
