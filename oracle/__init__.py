"""CPU oracle for brute-force incoherent dedispersion -- TEST INFRASTRUCTURE.

This package is the independent reference that the GPU library is checked
against.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the product path never does, and the oracle imports nothing
from the product package.  See ``oracle.c`` for what is computed and which
passage of the paper each part follows.
"""
from .oracle import (  # noqa: F401
    KDM,
    adjoint,
    bin_time,
    build,
    corner_turn,
    forward,
    forward_f32,
    lib_path,
    n_out_for,
    shift_table,
)
from .eq3_literal import eq3_literal, shift_literal  # noqa: F401
