"""CPU oracle for the ARTS single-pulse search hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct statement of what
the search computes, used to check the HIP library.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import it; the
product package ``paper_2205_12362_amd`` never does, and shares no code with it.
"""
from .arts_oracle import *  # noqa: F401,F403
