"""TEST INFRASTRUCTURE ONLY: plain FP64 CPU oracle of the shaped-EOS pseudopotential LBM.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  It shares no code with the HIP product path.
"""
from .oracle import *  # noqa: F401,F403
