"""MI355X-native systolic 3D Yee FDTD (hand-written HIP for gfx950 behind a C ABI).

Submodules are imported lazily: ``workloads`` draws seeded inputs and has no
dependency on the compiled library; ``fdtd`` is the thin ctypes binding over
``libfdtd.so`` and fails loudly if the library has not been built.
"""
