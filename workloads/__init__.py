"""Seeded synthetic inputs shared by the CPU oracle, the GPU tests and the benchmark.

This package only draws inputs (frequency sets, lattice sizes and generating vectors for the
standalone transforms, sample vectors, planted sparse polynomials).  It holds none of the
method's arithmetic: no residues, no alias counting, no transforms and no detection logic.
"""
from .gen import *  # noqa: F401,F403
