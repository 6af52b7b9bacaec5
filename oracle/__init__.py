"""CPU oracle for the D2Q9 lattice-Boltzmann method of arXiv:2006.12910.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library; the library never imports it.
"""
from .oracle import (Oracle, OracleParams, normals, normals_bulk, own_logf,  # noqa: F401
                     own_sincos2pi, philox4x32_10)
