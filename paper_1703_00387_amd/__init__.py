"""MI355X (gfx950) two-site MPS update: TEBD gates and FP64 truncated SVD.

The compute path is libmps.so (HIP kernels behind a C ABI, include/mps.h);
this package only binds it.  Build with ``python -m paper_1703_00387_amd.build``.
"""
from ._lib import EXPORTS, LIB_PATH, MPSError, lib  # noqa: F401
