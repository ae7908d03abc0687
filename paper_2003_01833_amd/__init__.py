"""MI355X-native barycentric Lagrange treecode for the Green-function convolutions
of treecode-accelerated Green Iteration (arXiv 2003.01833).

The computation lives in libtagi.so (HIP kernels for gfx950 behind the C ABI of
include/tagi.h); ``binding`` marshals torch tensors into it.
"""
from .binding import (COULOMB, COULOMB_SS, FP64, MIXED, YUKAWA, YUKAWA_SS, TagiError, Tree,  # noqa: F401
                      autotune, autotune_cached, autotune_learned, direct, load_library, mesh,
                      treecode)
