"""CPU FP64 oracle (test infrastructure only).

Plain NumPy/SciPy implementations of what the GPU library computes, written
from the paper's equations.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` use it; the library never imports it.
"""
from . import multislice, rotation, adam  # noqa: F401
