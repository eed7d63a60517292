"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package draws numbers and lays them out; it performs none of the
coupled-cluster arithmetic (no contraction, no denominator, no energy).
Both the CPU oracle and the device path consume exactly the arrays built
here, so the two sides see bit-identical inputs.
"""
from .synth import (  # noqa: F401
    BASE_SEED,
    CCSystem,
    make_system,
    orbital_energies,
    pair_gaussian,
    splitmix64,
)
