"""FP64 CPU oracle for the LLG hot path (test infrastructure only).

This package is the slow, plain reference against which the HIP path is
checked.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product library never does, and the two
share no code.  Everything here runs in float64 with NumPy/SciPy.

Modules
-------
newell   demagnetising tensor of rectangular cells (Section II-B, Eq. (3))
demag    zero-padded FFT convolution and the O(N^2) direct sum it must equal
field    effective field: exchange, DMI with its boundary condition,
         anisotropy, Zeeman (Section II-A, Eqs. (2), (5), (7), (9), (10))
llg      LLG right-hand side, per-cell renormalisation, RK4, energy
         (Section II-A Eq. (1); Section II-B; Section III-C)
adjoint  hand-derived vector-Jacobian products of the above and a
         checkpointed reverse sweep over RK4 steps
"""
from .params import Grid, Params, TERM_DEMAG, TERM_EXCH, TERM_DMI, TERM_ANIS, TERM_ZEEMAN, TERM_ALL  # noqa: F401
