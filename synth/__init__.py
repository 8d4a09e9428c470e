"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle's tests.

This module holds no Gray-Scott arithmetic: only parameter sets (the problem
constants of the paper's Section 3.1 and its provenance record, Listing 1) and
seeded random draws (random states, random (F, k) sweeps, random blob
placements). Whatever the method computes from these inputs is implemented
separately by the oracle and by the HIP library.
"""
from .inputs import *  # noqa: F401,F403
