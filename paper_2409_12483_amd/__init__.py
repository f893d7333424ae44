"""MI355X-native ADER-DG / ADER-WENO-FV hot path (1-D).

The compute lives in the HIP library ``libaderdg.so`` (built from
``csrc/``); ``abi`` is a thin ctypes binding with the same entry-point
names as ``include/aderdg.h``.  Importing this package does not load the
library; ``abi.load()`` does, and fails loudly if it is missing.
"""
