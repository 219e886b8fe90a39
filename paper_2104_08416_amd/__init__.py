"""MI355X-native Hilbert-ordered spectral-element time step (2D acoustic, GLL quads).

The compute path is the HIP library ``libsem_hip.so`` behind the C ABI of
``include/sem.h``; ``sem`` is its ctypes binding. Importing ``sem`` fails loudly when the
library has not been built (``python -m paper_2104_08416_amd.build``).
"""
__all__ = ["sem", "build"]
