"""MI355X-native spectral-element Poisson operator and Jacobi-PCG.

The compute path is libsem.so (hand-written HIP for gfx950 behind the C ABI of
include/sem.h); this package holds its build script and a thin binding that
takes device memory and streams from PyTorch.
"""

from ._lib import LIB_PATH, SemError  # noqa: F401
from .sem import (ASSEMBLED, LOCAL, MASKED, OP_TILE, UPDATE_TILE, CgResult, SemOperator,  # noqa: F401
                  knob_count, mesh_desc,
                  gs, gs_csr_build, vec_axpy, vec_axpy_generic, vec_dot, vec_dot_generic,
                  vec_dot_noalloc, vec_dot_workspace, workspace_bytes)
