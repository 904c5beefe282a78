"""seisgrad on MI355X: explicit finite-difference wave propagation with PML,
source injection, receiver gathering and the exact adjoint (misfit gradient),
as hand-written HIP kernels for gfx950 behind a small C ABI.

Importing the package loads nothing; the native library is opened by
:mod:`paper_2003_06027_amd.seisgrad` on first use and fails loudly when it
has not been built.
"""
