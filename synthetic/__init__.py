"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  This package holds no arithmetic of the finite-volume method:
it only synthesises fields (real spherical harmonics, uniform noise) at the
node coordinates the caller passes in, plus their closed-form derivatives,
which the convergence tests use as the analytic truth."""
from .sh_fields import (  # noqa: F401
    SHCoeffs, random_coeffs, synthesize, synthesize_gradient, laplacian_coeffs,
    rotated_gradient, config_field, level_field_stack, noise, seed_rng,
)
