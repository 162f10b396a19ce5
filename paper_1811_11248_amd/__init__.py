"""MI355X (gfx950) deferred-compression hierarchical solver.

The factorization, substitution sweeps and PCG run in hand-written HIP
kernels behind the C interface of ``include/lrsp.h`` (``liblrsp.so``);
``lrsp`` is the ctypes binding.  Loading fails loudly when the library has
not been built (``python -m paper_1811_11248_amd.build``).
"""
from .lrsp import (  # noqa: F401
    DeviceMatrix,
    Factor,
    LrspError,
    Tree,
    apply,
    factor,
    lib,
    pcg,
    tree_build,
)
