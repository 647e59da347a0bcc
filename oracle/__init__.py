"""Plain FP64 CPU oracle for the TT hot path.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` (the CPU part of a bench run, after the GPU
lines: it times this oracle on the host and checks the headline result and
sampled serving requests against it) are the only callers.  It shares no code
with the HIP library and never imports it.

Parity pins: every function here is checked by ``tests/test_oracle_*.py``
against dense brute force, closed forms and invariants.
"""
from .tt import *          # noqa: F401,F403
from .schemes import *     # noqa: F401,F403
from . import dense        # noqa: F401
from .laplace import *     # noqa: F401,F403
from .randomized import *  # noqa: F401,F403
