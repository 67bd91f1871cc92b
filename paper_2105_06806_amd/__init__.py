"""MI355X-native exact-diagonalisation hot path (arXiv 2105.06806).

Submodules:
  edx     -- ctypes binding of the HIP library libedx.so (C ABI in include/edx.h)
  inputs  -- seeded synthetic Anderson-impurity inputs
  build   -- hipcc build of libedx.so for gfx950
The binding is imported on demand (``from paper_2105_06806_amd import edx``) so
that the input generator can be used without torch or the library.
"""
