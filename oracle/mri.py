"""Explicit-explicit multirate (MRI) time stepping of Eq. (1) (FP64 oracle).

Test infrastructure only.

Section III-C (integrator comparison on Standard Problem 4) splits the
right-hand side additively into a fast part, the LLG torque of the exchange
field alone, and a slow part, the torque of every other term (demag, DMI,
anisotropy, bias).  Eq. (1) is linear in H for fixed m, so
R(m) = R(m, H_exch) + R(m, H_eff - H_exch) exactly.  Both time scales use the
three-stage third-order explicit method of Knoth and Wolke; the slow step is
dt and the fast step is a tenth of it.

Multirate infinitesimal step (MIS) form of the method (Knoth and Wolke 1998;
the MRI-GARK family of Sandu 2019 contains it): with slow Butcher table
(A, b, c), s = 3 stages, and the extra row a_{s+1} = b, c_{s+1} = 1,
  Y_1 = y_n
  for i = 2 .. s+1: v(0) = Y_{i-1};
      dv/dtau = f_F(v) + (1 / dc_i) sum_j (a_ij - a_{i-1,j}) f_S(Y_j),
      tau in [0, dc_i dt], dc_i = c_i - c_{i-1};   Y_i = v(dc_i dt)
  y_{n+1} = Y_{s+1}.
The fast ODE of each interval is integrated with the same Knoth-Wolke
table in n_i equal substeps, n_i the smallest integer with
n_i dt_fast >= dc_i dt (1 - 1e-12).

Readings (the paper gives neither):
* Knoth-Wolke table: c = (0, 1/3, 3/4); A and b are the unique solution of
  the third-order conditions for these nodes (solved below in exact rational
  arithmetic), which is the published method.
* Substeps of equal length per interval (a fixed fast step with a shortened
  last substep converges to the same limit).
* Renormalisation (Section II-B) with renorm = 2: every slow stage value
  Y_2, Y_3 and the new state; renorm = 1: the new state only; fast substeps
  are not renormalised.
"""
from dataclasses import replace
from fractions import Fraction as Fr
import math

import numpy as np

from . import field
from .llg import normalize, rhs_from_field
from .params import TERM_DMI, TERM_EXCH

KW3_C = (Fr(0), Fr(1, 3), Fr(3, 4))


def kw3_table():
    """(A, b, c) of the Knoth-Wolke method as Fractions: a21 = c2,
    a31 + a32 = c3, and b, a32 from the four third-order conditions
      sum b = 1, sum b c = 1/2, sum b c^2 = 1/3, b3 a32 c2 = 1/6."""
    c1, c2, c3 = KW3_C
    # b2 c2 + b3 c3 = 1/2 and b2 c2^2 + b3 c3^2 = 1/3 (2x2 linear system)
    det = c2 * c3 * c3 - c3 * c2 * c2
    b2 = (Fr(1, 2) * c3 * c3 - Fr(1, 3) * c3) / det
    b3 = (Fr(1, 3) * c2 - Fr(1, 2) * c2 * c2) / det
    b1 = 1 - b2 - b3
    a32 = Fr(1, 6) / (b3 * c2)
    A = ((Fr(0), Fr(0), Fr(0)), (c2, Fr(0), Fr(0)), (c3 - a32, a32, Fr(0)))
    return A, (b1, b2, b3), (c1, c2, c3)


def _float_table():
    A, b, c = kw3_table()
    return [[float(v) for v in row] for row in A], [float(v) for v in b], [float(v) for v in c]


def erk_step(f, y, h):
    """One step of the Knoth-Wolke explicit RK method for y' = f(y)."""
    A, b, _ = _float_table()
    ks = []
    for i in range(3):
        yi = y
        for j in range(i):
            yi = yi + h * A[i][j] * ks[j]
        ks.append(f(yi))
    out = y
    for i in range(3):
        out = out + h * b[i] * ks[i]
    return out


def substeps(dc, dt, dt_fast):
    """Number of equal fast substeps covering dc*dt with steps <= dt_fast."""
    return max(1, int(math.ceil(dc * dt / dt_fast * (1.0 - 1e-12))))


def mis_step(f_fast, f_slow, y, dt, dt_fast, stage_map=None, slow_time=False):
    """One MIS step of the Knoth-Wolke pair for y' = f_fast(y) + f_slow(y).
    stage_map (optional) is applied to each slow stage value Y_2..Y_{s+1}
    (renormalisation).  With slow_time, f_slow(Y, c) also receives the node
    c_i of the slow stage (non-autonomous slow part, e.g. a time-dependent
    bias field).  Returns (y_{n+1}, slow stage values, fast evaluations)."""
    A, b, c = _float_table()
    Arows = A + [b]
    cc = c + [1.0]
    Y = [y]
    S = []
    nfast = 0
    for i in range(1, 4):
        S.append(f_slow(Y[i - 1], cc[i - 1]) if slow_time else f_slow(Y[i - 1]))
        dc = cc[i] - cc[i - 1]
        r = 0.0
        for j in range(i):
            r = r + (Arows[i][j] - Arows[i - 1][j]) / dc * S[j]
        n = substeps(dc, dt, dt_fast)
        h = dc * dt / n
        v = Y[i - 1]
        for _ in range(n):
            v = erk_step(lambda u: f_fast(u) + r, v, h)
            nfast += 3
        if stage_map is not None:
            v = stage_map(v)
        Y.append(v)
    return Y[3], Y, nfast


def split_fields(grid, p, m, spec=None, pshape=None):
    """(H_exch, H_eff - H_exch) of m with the ghost rule of the full field."""
    parts = field.heff_parts(grid, p, m, spec, pshape)
    hf = parts.get("exch", np.zeros(np.shape(m)))
    hs = np.zeros(np.shape(m))
    for k, v in parts.items():
        if k != "exch":
            hs = hs + v
    return hf, hs


def fast_rhs(grid, p, m):
    """Torque of the exchange field alone (no FFT), with the boundary rule of
    the full field (the DMI condition of Eq. (10) and, with a magnetisation
    profile, the surface of the magnet)."""
    if not p.has(TERM_EXCH):
        return np.zeros(np.shape(m))
    if getattr(p, "ms_profile", None) is not None:
        q = replace(p, terms=p.terms & (TERM_EXCH | TERM_DMI))
        return rhs_from_field(p, m, field.heff_parts_masked(grid, q, np.asarray(m, np.float64))["exch"])
    g = field.ghost_padded(grid, p, m)
    return rhs_from_field(p, m, field.exchange(grid, p, m, g))


def slow_rhs(grid, p, m, spec=None, pshape=None):
    """Torque of H_eff - H_exch (demag, DMI, anisotropy, bias)."""
    _, hs = split_fields(grid, p, m, spec, pshape)
    return rhs_from_field(p, m, hs)


def mri_step(grid, p, m, dt, dt_fast, spec=None, pshape=None, t0=0.0, bias_at=None):
    """One multirate step of the LLG equation.  Returns (m_{n+1}, number of
    slow evaluations, number of fast evaluations).  With bias_at (time ->
    H_bias), slow stage i sees the bias at t0 + c_i dt."""
    from .llg import with_bias
    m = np.asarray(m, dtype=np.float64)
    stage_map = (lambda v: normalize(v)[0]) if p.renorm == 2 else None
    if bias_at is None:
        f_slow = lambda u, c: slow_rhs(grid, p, u, spec, pshape)  # noqa: E731
    else:
        f_slow = lambda u, c: slow_rhs(grid, with_bias(p, bias_at(t0 + c * dt)), u, spec, pshape)  # noqa: E731
    out, _, nfast = mis_step(lambda u: fast_rhs(grid, p, u), f_slow, m, dt, dt_fast, stage_map, slow_time=True)
    if p.renorm >= 1 and stage_map is None:
        out = normalize(out)[0]
    return out, 3, nfast


def mri_run(grid, p, m, dt, dt_fast, nsteps, spec=None, pshape=None, t0=0.0, bias_at=None):
    for n in range(nsteps):
        m = mri_step(grid, p, m, dt, dt_fast, spec, pshape, t0 + n * dt, bias_at)[0]
    return m
