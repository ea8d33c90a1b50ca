"""MI355X (gfx950) library for the contour-integral sign function and the
overlap-Dirac operator of Nagai & Tomiya (arXiv:2204.01583).

The work is done by the HIP library ``libovl.so`` (C ABI in include/ovl.h);
``paper_2204_01583_amd.ovl`` is a thin ctypes binding over it.  Importing
this package loads nothing; ``paper_2204_01583_amd.ovl.load()`` loads the
library and raises if it has not been built.
"""

__all__ = ["ovl", "build"]
