"""Chunked-SVDAG primary-ray traversal on MI355X (HIP for gfx950).

- ``svdag``: ctypes binding of ``libsvdag.so`` (the C ABI of
  ``include/svdag.h``): DAG build, world residency, per-view and batched
  traces, and the request server.
- ``scenes``: seeded synthetic scenes, camera poses and request loads (inputs
  only; no traversal arithmetic).
- ``build``: compiles the library in place.
"""
