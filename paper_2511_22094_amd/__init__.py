"""MI355X-native voxel-parallel model fitting (Metropolis-Hastings / ensemble
MCMC and Adam-type whole-volume fits) behind the C ABI of include/gacelle.h.

``synth`` (seeded synthetic inputs) imports without the compiled library;
``lib()`` loads the HIP library and fails loudly if it has not been built.
"""

__all__ = ["lib", "synth"]


def lib():
    """The ctypes binding of libgacelle.so (raises ImportError if not built)."""
    from . import _lib
    return _lib
