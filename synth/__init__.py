"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package only draws random numbers and lays them out in the canonical
formats of the library boundary. It holds none of the method's arithmetic (no
Dirac operator, solver, force or integrator), so both sides of a parity test can
consume the same arrays without sharing any computation.
"""
from .fields import (  # noqa: F401
    SEED_BASE,
    make_rng,
    random_su3_near_identity,
    haar_su3,
    gaussian_half_vector,
    gaussian_momentum,
    lattice_volume,
    load_rational,
)
