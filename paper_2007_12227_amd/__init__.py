"""MI355X-native phase-space-conservation Vlasov solver (push + re-deposit + mass-matrix solve).

The compute path is the HIP library ``libvp.so`` (built from ``csrc/``) behind
the C interface ``include/vp.h``; ``binding`` is its ctypes wrapper.  Importing
this package loads nothing; ``binding.lib()`` loads the library and raises if
it has not been built.
"""
__all__ = ["inputs"]
