"""MI355X-native semisort, histogram and collect-reduce (Dong et al., SPAA 2023).

The hot path runs as hand-written HIP kernels for gfx950 behind the C-ABI
library ``libsemisort_hip.so`` (declared in ``include/semisort.h``).  The
Python layer in :mod:`paper_2304_10078_amd.semisort` only marshals arguments.
"""
__all__ = ["semisort", "inputs"]
