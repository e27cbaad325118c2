"""MI355X-native Kohn-Sham direct minimisation on the Stiefel manifold.

Hot path in HIP (``csrc/``, built into ``libks.so``) behind the C ABI of
``include/ks.h``; ``ks`` is the ctypes binding (loaded on first import of that
module, and it fails loudly when the library is missing); ``synth`` draws the
seeded synthetic inputs.
"""
__all__ = ["synth"]
