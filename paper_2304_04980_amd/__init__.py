"""MI355X (gfx950) solver for LQ optimal control over 2D grids by NBJM-
preconditioned conjugate gradients (Zafar & Manchester, arXiv 2304.04980).

The compute path is liblqgrid.so (hand-written HIP, C ABI in include/lqgrid.h);
``paper_2304_04980_amd.lqgrid`` is its Python binding.
"""
