"""FP64 CPU oracle for PCG map-making with block-diagonal and two-level
preconditioners (Puglisi et al. 2018, arXiv:1801.08937).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the GPU library computes, used to check it.  Only the test
suite, the smoke entry point and the benchmark's CPU-baseline leg may import
it.  The GPU library never calls it, and it shares no code with the GPU
library: the only common module is ``synth`` (seeded input generation).

Every function cites the passage of the paper it follows; readings of points
the paper leaves open are stated where they are used.
"""
from .mapmaking import *  # noqa: F401,F403
