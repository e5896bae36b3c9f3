"""CPU FP64 reference implementations (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP library never calls it.
"""
from . import lshom_oracle  # noqa: F401
