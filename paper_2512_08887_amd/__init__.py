"""MI355X (gfx950) fast broadband beamspace transformation.

libfbst.so (C ABI in include/fbst.h, HIP kernels in csrc/) does all the work;
``fbst`` is its ctypes binding.  Importing this package loads nothing: the
library is opened on first use and must have been built
(``python -m paper_2512_08887_amd.build``).
"""
__all__ = ["fbst"]
