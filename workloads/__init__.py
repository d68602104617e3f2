"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This package holds only the random draws that define an instance (coupling
matrix, clause list, weights) and its starting points, plus the paper's
hyper-parameter table.  It contains none of the method's arithmetic: neither the
oracle under ``oracle/`` nor the HIP library imports anything else in common.
"""
from .gen import *  # noqa: F401,F403
from .params import *  # noqa: F401,F403
