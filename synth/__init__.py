"""Seeded synthetic input generators shared by the tests, the benchmark and
the oracle.  Holds random-number and input-recipe code only."""
from . import rng, problems  # noqa: F401
