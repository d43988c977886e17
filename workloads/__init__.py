"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's checks.

This module draws random fields, ensembles and observations only; it holds no part of
the filter's arithmetic, so that the GPU path and the CPU oracle stay independent.
"""
from .fields import smooth_field, smooth_fields, field_psd_slope
from .configs import (Problem, make_problem, config_problem, batched_problems,
                      CONFIG_SEEDS, config_shapes)

__all__ = ["smooth_field", "smooth_fields", "field_psd_slope", "Problem", "make_problem",
           "config_problem", "batched_problems", "CONFIG_SEEDS", "config_shapes"]
