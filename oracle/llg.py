"""LLG right-hand side, renormalisation, classical RK4 and energy (FP64 oracle).

Test infrastructure only.

* Eq. (1) for unit m (M = Ms m):  dm/dt = R(m) = a [m x H + alpha m x (m x H)],
  a = mu0 gamma_L, gamma_L = gamma / (1 + alpha^2), gamma = -1.759e11 as printed.
* Renormalisation (Section II-B): after each time step or stage evaluation
  |m| is reset to 1 in every cell.  Reading used here (mode 2): every stage
  input y2, y3, y4 and the new state are renormalised; y1 is the state as
  given.  Mode 1 renormalises only the new state, mode 0 never.
* Classical RK4 with fixed dt and four right-hand-side evaluations per step
  (Section III-C and its integrator comparison table): c = (0, 1/2, 1/2, 1),
  b = (1/6, 1/3, 1/3, 1/6).
* Energy: sum of the densities of Eqs. (4), (6), (8), the DMI density whose
  variational derivative is Eq. (9), and the Zeeman density.  Because
  H_eff = K m + H_bias with K symmetric, the total equals
  sum_i V [-(mu0 Ms / 2) m_i . (H_eff,i + H_bias)] + N V Ku.  Eq. (4) as
  printed lacks the factor Ms; the dimensionally consistent -(mu0 Ms/2) m.H
  is used.
"""
import numpy as np

from . import field
from .params import TERM_ANIS, TERM_ZEEMAN


def cross(a, b):
    return field._cross(a, b)


def dot(a, b):
    return np.sum(a * b, axis=0)


def prefactor(p):
    """a = mu0 * gamma / (1 + alpha^2)."""
    return p.mu0 * p.gamma / (1.0 + p.alpha * p.alpha)


def rhs_from_field(p, m, H):
    a = prefactor(p)
    mxH = cross(m, H)
    return a * (mxH + p.alpha * cross(m, mxH))


def rhs(grid, p, m, spec=None, pshape=None):
    return rhs_from_field(p, m, field.heff(grid, p, m, spec, pshape))


def normalize(x):
    """Per-cell x/|x|; a zero vector is left unchanged."""
    n = np.sqrt(dot(x, x))
    safe = np.where(n > 0, n, 1.0)
    return x / safe[None], n


RK4_C = (0.0, 0.5, 0.5, 1.0)
RK4_B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)


def rk4_step(grid, p, m, dt, spec=None, pshape=None, record=None):
    """One classical RK4 step.  If `record` is a list, the stage inputs y_s,
    fields H_s, pre-normalisation vectors x_s and their norms are appended."""
    stage_norm = p.renorm == 2
    m = np.asarray(m, dtype=np.float64)
    y = m
    ks = []
    xs = [None]
    ys = [m]
    Hs = []
    for s in range(4):
        H = field.heff(grid, p, y, spec, pshape)
        k = rhs_from_field(p, y, H)
        Hs.append(H)
        ks.append(k)
        if s < 3:
            x = m + RK4_C[s + 1] * dt * k
            y = normalize(x)[0] if stage_norm else x
            xs.append(x)
            ys.append(y)
    x5 = m + dt * sum(b * k for b, k in zip(RK4_B, ks))
    out = normalize(x5)[0] if p.renorm >= 1 else x5
    if record is not None:
        record.append(dict(y=ys, H=Hs, x=xs + [x5], out=out))
    return out


def energy_parts(grid, p, m, spec=None, pshape=None):
    """Per-term energies (J): demag, exch, dmi, anis, zeeman, and total."""
    parts = field.heff_parts(grid, p, m, spec, pshape)
    V = grid.volume
    out = {}
    for name, H in parts.items():
        e = -0.5 * p.mu0 * p.Ms * V * float(np.sum(m * H))
        if name == "zeeman":
            e *= 2.0
        if name == "anis":
            e += grid.ncell * V * p.Ku
        out[name] = e
    out["total"] = sum(out.values())
    return out


def energy(grid, p, m, spec=None, pshape=None):
    """Closed form of the total: sum V[-(mu0 Ms/2) m.(H_eff + H_bias)] + N V Ku."""
    H = field.heff(grid, p, m, spec, pshape)
    V = grid.volume
    h = np.zeros(3) if not p.has(TERM_ZEEMAN) else np.asarray(p.Hbias, np.float64)
    e = -0.5 * p.mu0 * p.Ms * V * float(np.sum(m * (H + h.reshape(3, 1, 1, 1))))
    if p.has(TERM_ANIS):
        e += grid.ncell * V * p.Ku
    return e
