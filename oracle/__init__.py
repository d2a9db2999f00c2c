"""CPU oracle for IVF-RaBitQ search — TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy statement of what the search path computes, written
from the paper (Sections 2.1-2.2 and 3.1). Only the test suite, the smoke check
of ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
it. The GPU library never calls it, and the two share no code: the oracle takes
its inputs from the ``synth`` generators or from the caller, never from the GPU
path.

Parity pins: every function below is pinned by ``-m "not gpu"`` tests against
closed forms, brute force, exact rational arithmetic or hand-computed fixtures
(see tests/test_oracle_*.py). No function is "parity unpinned".
"""
from .rabitq import *  # noqa: F401,F403
