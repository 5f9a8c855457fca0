"""MI355X-native block orthogonalisation (TreeTSPQR with BCGS-PIP+ leaves).

The compute path is liborth.so (HIP kernels for gfx950, C ABI in
include/orth.h); ``orth`` is its ctypes binding.  Build the library with
``python -m paper_2204_13393_amd.build``.
"""

from . import autotune, orth  # noqa: F401
from .orth import BatchOrthogonalizer, Orthogonalizer, OrthError, laplacian_apply, load  # noqa: F401

__all__ = ["autotune", "orth", "Orthogonalizer", "BatchOrthogonalizer", "OrthError", "laplacian_apply", "load"]
