"""MI355X (gfx950) KADABRA adaptive-sampling betweenness approximation.

The sampling path runs in the HIP library ``libkadabra_hip.so`` behind the
C-ABI in ``include/kadabra.h``; ``paper_1910_11039_amd.kadabra`` is its
Python binding (argument marshalling only).
"""

__all__ = ["kadabra"]
