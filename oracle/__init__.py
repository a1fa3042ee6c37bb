"""CPU oracle of the ideal-MHD update (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never uses it.
"""
from .oracle import *  # noqa: F401,F403
