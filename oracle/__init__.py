"""CPU oracle for the micro-macro parareal hot path (arXiv 1912.09240).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import anything from this package.  It
is a plain, slow restatement of the method (scalar C loops for the particles,
numpy for the rest, FP64 throughout) and shares no code with the HIP library.
"""
from . import coarse, iterate, particles, restrict  # noqa: F401
