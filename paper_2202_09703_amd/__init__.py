"""MI355X (gfx950) library for multi-layer, collimated-beam ultrasound MBIR
(arXiv:2202.09703): the matrix-free system matrix, its transpose and MAP
reconstruction, as hand-written HIP kernels behind the C ABI in
include/umbir.h.  `umbir` is the Python binding; `build` compiles the library.
"""
