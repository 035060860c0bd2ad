"""FP64 CPU oracle for the propagation hot path -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library.
"""
from .optics import *  # noqa: F401,F403
from .lattice import *  # noqa: F401,F403
