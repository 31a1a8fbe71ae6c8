"""FP64 CPU oracle of the DPM score-estimation path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does.
"""
from .dpm import *  # noqa: F401,F403
from . import dpm  # noqa: F401
