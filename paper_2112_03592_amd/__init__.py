"""MI355X-native discrete convolution on Adaptive Particle Representations.

The compute path is the HIP library ``libaprconv.so`` (C ABI in
``include/aprconv.h``); ``apr`` is its Python binding.  Importing the package
does not load the library; the first call that needs it does, and fails
loudly if it is not built.
"""

__all__ = ["apr"]
