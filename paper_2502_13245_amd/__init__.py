"""MI355X-native range retrieval over graph indices.

The search runs in the HIP library built from ``csrc/`` (``librr.so``) behind
the C ABI in ``include/rr.h``; ``rr`` is its Python binding.
"""
__all__ = ["rr", "synth", "build_lib"]
