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
* Forward Euler (the integrator of the paper's scaling runs) and a
  time-dependent uniform bias H_bias(t) (piecewise linear in time), the bias
  of each stage taken at that stage's time.
* Energy: sum of the densities of Eqs. (4), (6), (8), the DMI density whose
  variational derivative is Eq. (9), and the Zeeman density.  Because
  H_eff = K m + H_bias with K symmetric, the total equals
  sum_i V [-(mu0 Ms / 2) m_i . (H_eff,i + H_bias)] + N V Ku.  Eq. (4) as
  printed lacks the factor Ms; the dimensionally consistent -(mu0 Ms/2) m.H
  is used.
"""
from dataclasses import replace

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


def bias_schedule(times, values):
    """Time-dependent uniform bias field (NEXT row f3): piecewise-linear
    interpolation of the (time, H) knots, held constant before the first and
    after the last knot.  Returns t -> H (3,)."""
    times = np.asarray(times, dtype=np.float64)
    values = np.asarray(values, dtype=np.float64).reshape(-1, 3)

    def at(t):
        return np.array([np.interp(t, times, values[:, c]) for c in range(3)])
    return at


def with_bias(p, h):
    return replace(p, Hbias=tuple(float(v) for v in h))


def euler_step(grid, p, m, dt, spec=None, pshape=None, t0=0.0, bias_at=None):
    """Forward Euler (used by the paper for its weak-scaling runs):
    m_{n+1} = m_n + dt R(m_n), renormalised when renorm >= 1.  With bias_at,
    H_bias is taken at the step's start time t0."""
    m = np.asarray(m, dtype=np.float64)
    q = with_bias(p, bias_at(t0)) if bias_at is not None else p
    x = m + dt * rhs(grid, q, m, spec, pshape)
    return normalize(x)[0] if p.renorm >= 1 else x


def rk4_step(grid, p, m, dt, spec=None, pshape=None, record=None, t0=0.0, bias_at=None):
    """One classical RK4 step.  If `record` is a list, the stage inputs y_s,
    fields H_s, pre-normalisation vectors x_s and their norms are appended.
    With bias_at (time -> H_bias), stage s sees the bias at t0 + c_s dt."""
    stage_norm = p.renorm == 2
    m = np.asarray(m, dtype=np.float64)
    y = m
    ks = []
    xs = [None]
    ys = [m]
    Hs = []
    for s in range(4):
        ps = with_bias(p, bias_at(t0 + RK4_C[s] * dt)) if bias_at is not None else p
        H = field.heff(grid, ps, y, spec, pshape)
        k = rhs_from_field(ps, y, H)
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
    # Ms of every cell (space-dependent with a profile; 0 outside the magnet)
    s = np.ones(grid.shape) if getattr(p, "ms_profile", None) is None else np.asarray(p.ms_profile, np.float64)
    out = {}
    for name, H in parts.items():
        e = -0.5 * p.mu0 * p.Ms * V * float(np.sum(s[None] * m * H))
        if name == "zeeman":
            e *= 2.0
        if name == "anis":
            e += float(np.count_nonzero(s > 0)) * V * p.Ku
        out[name] = e
    out["total"] = sum(out.values())
    return out


def energy(grid, p, m, spec=None, pshape=None):
    """Closed form of the total: sum V[-(mu0 Ms/2) m.(H_eff + H_bias)] + N V Ku."""
    if getattr(p, "ms_profile", None) is not None:
        return energy_parts(grid, p, m, spec, pshape)["total"]
    H = field.heff(grid, p, m, spec, pshape)
    V = grid.volume
    h = np.zeros(3) if not p.has(TERM_ZEEMAN) else np.asarray(p.Hbias, np.float64)
    e = -0.5 * p.mu0 * p.Ms * V * float(np.sum(m * (H + h.reshape(3, 1, 1, 1))))
    if p.has(TERM_ANIS):
        e += grid.ncell * V * p.Ku
    return e
