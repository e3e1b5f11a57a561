"""Seeded synthetic inputs (molecules, Cartesian shells, factor parameters).

This module holds no arithmetic of the integral method: it only draws
geometries, exponents and coefficients.  Both the CPU oracle's tests and the
GPU library's tests/benchmarks take their inputs from here.
"""
from .molecules import (Factor, FACTOR_SETS, GENERIC_FACTORS, Shell, molecule, tiny_config,
                        config_plain, config_batching_extra, config_precision,
                        shells_to_arrays)
