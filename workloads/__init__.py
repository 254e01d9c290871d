"""Seeded synthetic NNLS instances shared by the oracle side and the GPU side.

This module only draws random numbers and assembles ``b = A x_true + noise``;
it holds none of the solver's arithmetic.  Both the CPU oracle and the HIP path
receive byte-identical inputs from it.
"""
from .generators import (  # noqa: F401
    Instance,
    make_gaussian_planted,
    make_c1,
    make_c2,
    make_c3,
    make_c4_batch,
    make_c4_instance,
    make_c5_batch,
    make_small,
    make_illcond,
    make_signed,
    CONFIGS,
)
