"""FP64 CPU oracle (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
