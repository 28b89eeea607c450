"""FP64 CPU oracle for the spin-2 QLG step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path.
"""
from .qlg_oracle import *  # noqa: F401,F403
from . import qlg_oracle  # noqa: F401
