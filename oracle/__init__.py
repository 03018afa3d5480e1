"""CPU FP64 reference of the particle-in-cell flavor method.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares no code with the HIP
library (see fpic_oracle.c for what it computes and why).
"""
from .oracle import ParticleProblem, Problem, set_threads  # noqa: F401
