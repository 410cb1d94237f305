"""Test infrastructure: the CPU double-precision oracle of the implicit step.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the GPU library.
"""
from .oracle import Oracle, build, tridiag, gmres_dense, lib_path, threads  # noqa: F401
