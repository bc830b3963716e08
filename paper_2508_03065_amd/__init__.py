"""msim: moving-source image-source synthesis on MI355X (gfx950).

The synthesis runs in libmsim.so (hand-written HIP kernels behind the C-ABI of
include/msim.h); the submodule `paper_2508_03065_amd.msim` marshals arguments
to it, `scenegen` describes seeded synthetic inputs.
"""
from . import scenegen  # noqa: F401
