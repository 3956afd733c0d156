"""MI355X-native matrix-free DG operators for scale-resolved Li-S cathodes.

The compute path lives in the HIP library ``liblsbdg.so`` (C-ABI declared
in include/lsbdg.h); ``lsbdg`` is a thin ctypes binding with the same entry
points that marshals torch device tensors and the current HIP stream.
Importing this package does not load the library; ``lsbdg.load()`` does and
raises if it is missing.
"""
