"""Oracle for GPS L1 C/A acquisition -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation of what the acquisition search computes
(the acquisition channel of the paper's Fig. 2, Sec. 3).  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
it.  It shares no code with the HIP library (``paper_1309_0052_amd``).

Every function states the passage it follows.  Parity pins are in
``tests/test_oracle_*.py``.  Functions without an independent pin say
"parity unpinned" in their docstring.
"""
from .oracle import *  # noqa: F401,F403
