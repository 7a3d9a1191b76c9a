"""MI355X-native twisted-mass disconnected-loop library.

The compute path lives in the HIP library ``_lib/libtm.so`` (kernels in
``csrc/``, C ABI in ``include/tm.h``); ``tm`` is its ctypes binding and
``inputs`` holds the seeded synthetic input generators.
"""
__all__ = ["tm", "inputs"]
