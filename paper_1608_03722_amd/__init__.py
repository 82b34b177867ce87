"""MI355X (gfx950) Langevin hot path of the single-nucleotide dsDNA model of
Fosado et al. (arXiv:1608.03722).  The computation lives in libdsdna.so
(C ABI in include/dsdna.h); `dsdna` is its ctypes binding."""
