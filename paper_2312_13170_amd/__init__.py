"""Loop-internalised contraction kernels for MI355X (gfx950).

GEMM, the two-GEMM chain, covariance and correlation as hand-written HIP
kernels behind a C ABI (libli.so); this package holds the kernels' sources
(csrc/), the build script and a thin ctypes binding (li.py) with the same
entry-point names as the C header.  Importing the package loads nothing;
`from paper_2312_13170_amd import li` loads the library and fails loudly if
it has not been built.
"""
