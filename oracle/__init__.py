"""CPU oracle for the D2Q9 lattice-Boltzmann method of arXiv:2006.12910.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library; the library never imports it.
"""
from .oracle import Oracle, OracleParams, philox4x32_10, normals, own_logf, own_sincos2pi  # noqa: F401
