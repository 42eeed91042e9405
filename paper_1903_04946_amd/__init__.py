"""MI355X (gfx950) implementation of the composed split-operator propagator
of arXiv:1903.04946 for separable diabatic Hamiltonians.

The propagation runs in ``libsoprop.so`` (HIP kernels behind a C ABI,
``include/soprop.h``); ``soprop`` is its ctypes binding and ``synth`` holds
the seeded synthetic models.  Importing the package loads nothing; the
library is loaded on first use and its absence is an error.
"""

__all__ = ["soprop", "synth", "build"]
