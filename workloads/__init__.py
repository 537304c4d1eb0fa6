"""Seeded synthetic workloads for the Holstein fermion solve.

This package holds only parameters and random draws: phonon fields ``x``,
Gaussian pseudofermion draws ``phi`` and Rademacher measurement vectors
``xi``.  It contains none of the method's arithmetic, so that the CPU oracle
(``oracle/``) and the GPU path can both consume the same inputs without
sharing any computation.
"""

from .configs import CONFIGS, HmcParams, Params, get_config, hmc_params  # noqa: F401
from .inputs import (  # noqa: F401
    rng_for,
    phonon_field,
    gaussian_rhs,
    rademacher_rhs,
    perturbed_field,
    batched_systems,
    fd_sample_indices,
    hmc_draws,
)
