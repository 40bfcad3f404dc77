"""FP64 CPU oracle for the sampled Tucker core update (test infrastructure).

This package is the slow, plain reference the HIP library is checked against.
It is test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
GPU path (``paper_2107_10654_amd``) and never imports it.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against facts of the paper or of the mathematics (see the pin list in each
test module).
"""
from . import philox, tucker_ref  # noqa: F401
from .tucker_ref import *  # noqa: F401,F403
