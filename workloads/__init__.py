"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds input generators only (problem instances, MIMO detection
problems, annealing schedules and noise quantile tables).  It contains none of the update rule's
arithmetic, so the HIP path and the oracle can both take its outputs without
sharing any of the method's code.
"""
from .instances import sk1, maxcut, random_int8, dense_problem  # noqa: F401
from .schedules import (  # noqa: F401
    linear_beta, eta_sqrt_beta_over_5, paper_tanh_beta, conventional_eta, constant,
    mimo_eta, mimo_conventional_eta,
)
from .noise import gauss_table, uniform_table  # noqa: F401
from . import mimo  # noqa: F401
