"""CPU FP64 oracle for the triboelectric particle step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call anything in this package.  The product path
(``paper_2602_10761_amd``) never imports it and shares no code with it; the
only shared module is the seeded input generator
``paper_2602_10761_amd.workload``, which holds none of the step's arithmetic.
"""
from .tribo_oracle import *  # noqa: F401,F403
