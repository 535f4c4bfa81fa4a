"""MI355X (gfx950) implementation of the hot path of the 2D axisymmetric
implicit PIC/MCC model with equivalent-capacitance circuit coupling of
arXiv 2310.04957.  The method runs in libpic.so (HIP kernels behind the C ABI
of include/pic.h); ``pic.Pic`` is its Python binding."""
