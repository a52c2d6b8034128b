"""MI355X-native split-operator Dirac sweep (libdirac) -- Python side.

The hot path runs in libdirac.so (HIP, gfx950).  `libdirac` holds the ctypes
binding; `inputs` the seeded synthetic inputs.  Nothing is loaded at import
time, so the inputs can be used without a GPU or a built library.
"""
__all__ = ["libdirac", "inputs"]
