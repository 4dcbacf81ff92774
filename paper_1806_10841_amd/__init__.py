"""MI355X-native hot path of force-interpolation AdResS.

* ``libadres.so`` (built from ``csrc/`` by ``build.py``): HIP kernels for gfx950
  behind the C ABI of ``include/adres.h``.
* ``binding``: ctypes marshalling of that ABI over torch device tensors.
* ``inputs``: seeded synthetic workloads (placement and random numbers only).

Importing the package loads nothing; ``binding.load_library()`` does, and raises
if the library has not been built.
"""
__all__ = ["binding", "inputs", "build"]
