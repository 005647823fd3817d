"""MI355X-native integer matrix power A^p (binary exponentiation on HIP/MFMA).

Submodules:
  mpow    - ctypes binding of libmpow (include/mpow.h), plus torch helpers
  inputs  - seeded synthetic input generators
  build   - hipcc build of libmpow.so (gfx950)
"""
from . import inputs  # noqa: F401
