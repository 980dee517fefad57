"""FP64 CPU oracle for the pmCIMb quadrature sweep (TEST INFRASTRUCTURE ONLY).

This package is the checker, not the product.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  The GPU path
never calls it and shares no code with it: the two meet only in the seeded
input generators of the ``gen`` package.

Everything here is plain complex128 numpy/scipy, written step by step in the
order the paper gives them (Sections 2.1-2.2 and 3.2, eqs (2.3)-(2.4),
(2.6)-(2.8), (3.1)-(3.3)), so that each function can be checked against the
paper by eye.  Each function is pinned by tests against closed forms,
brute force or library routines (tests/test_oracle_*.py).
"""
from .nep import *  # noqa: F401,F403
from . import brute  # noqa: F401
from . import pmcima  # noqa: F401,E402
