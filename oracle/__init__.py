"""FP64 CPU oracle of the CAC lattice Boltzmann wetting step.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.  See
``oracle/cac_oracle.c`` for the method and its readings.
"""
from .oracle import *  # noqa: F401,F403
