"""Seeded, synthetic input generators shared by the oracle tests, the GPU
tests and the benchmark.

This package holds initial data only: closed-form profiles (the exact
solitary wave of the SGN equations and the paper's perturbed / Gaussian /
crossing families) and seeded random smooth fields.  It contains none of the
solver's arithmetic (no spectral derivatives, no elliptic solves, no time
stepping), so that the oracle and the HIP path stay independent.
"""
from .generators import (  # noqa: F401
    Box,
    SolitonParams,
    soliton_params,
    soliton_profile,
    line_soliton,
    perturbed_line_soliton,
    deformed_line_soliton,
    soliton_plus_gaussian,
    gaussian_hump,
    crossing_solitons,
    ENSEMBLE_GRIDS,
    ensemble_member,
    random_smooth_field,
    random_state,
    workload,
    WORKLOADS,
    perturbed_soliton_sweep,
    SWEEP_AMPLITUDES,
    SWEEP_WAVENUMBERS,
)
