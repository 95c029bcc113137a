"""MI355X (gfx950) implementation of the L2-norm regularized
incremental-stencil WENO scheme (Zhu & Hu, arXiv 1908.02464) for the
compressible Euler equations: HIP kernels behind a C ABI
(include/weno_l2is.h), with a thin ctypes binding in ``capi``."""
