"""MI355X-native LLG hot path: effective field (demag FFT convolution,
exchange, DMI, anisotropy, Zeeman), RK4 time stepping with renormalisation,
and its reverse mode, in hand-written HIP kernels behind a C ABI
(include/magx.h).  This package holds the in-tree build of libmagx.so and a
ctypes binding; there is no CPU fallback."""
from .magx import (  # noqa: F401
    ANIS, DEMAG, DMI, EXCH, F32, F64, ZEEMAN, Context, HeffFunction, MagxError, Rollout, heff, load,
    magx_sizes, make_grid, make_params)
