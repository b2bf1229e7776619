"""Hand-derived reverse mode of the RK4/LLG step (FP64 oracle, test infrastructure only).

The paper motivates differentiable simulation but prints no adjoint; this is
the exact reverse of the forward algorithm in oracle.llg, derived by hand.

With H = K y + h (K symmetric, see oracle.field.linear_part) and
R(y) = a [y x H + alpha y x (y x H)], the vector-Jacobian product for a
cotangent kappa of R is

    mu     = a [kappa x y + alpha y x (y x kappa)]                  (cotangent of H)
    ybar   = a [H x kappa + alpha (H (y.kappa) + kappa (y.H) - 2 y (H.kappa))] + K mu
    hbar  += sum over cells of mu.

For P(x) = x/|x| the Jacobian is symmetric: P'(x)^T l = (l - p (p.l)) / |x|.

The reverse of one step walks the stages backwards, accumulating into the
cotangent of m_n; stage s feeds stage s-1 through x_s = m_n + c_s dt k_{s-1}.
A rollout keeps m every `ckpt` steps and recomputes each segment before
reversing it.
"""
import numpy as np

from . import field, llg
from .llg import RK4_B, RK4_C, cross, dot


def vjp_rhs(grid, p, y, H, kappa, spec=None, pshape=None):
    """Returns (ybar, mu) for cotangent kappa of R(y) at field H = H_eff(y)."""
    a = llg.prefactor(p)
    al = p.alpha
    mu = a * (cross(kappa, y) + al * cross(y, cross(y, kappa)))
    yk = dot(y, kappa)[None]
    yH = dot(y, H)[None]
    Hk = dot(H, kappa)[None]
    ybar = a * (cross(H, kappa) + al * (H * yk + kappa * yH - 2.0 * y * Hk))
    ybar = ybar + field.linear_part(grid, p, mu, spec, pshape)
    return ybar, mu


def vjp_normalize(x, lam):
    pn, n = llg.normalize(x)
    safe = np.where(n > 0, n, 1.0)[None]
    return (lam - pn * dot(pn, lam)[None]) / safe


def rk4_step_vjp(grid, p, m, dt, lam_out, spec=None, pshape=None):
    """Given m_n and the cotangent of m_{n+1}, returns (cotangent of m_n, hbar)."""
    rec = []
    llg.rk4_step(grid, p, m, dt, spec, pshape, record=rec)
    r = rec[0]
    ys, Hs, xs = r["y"], r["H"], r["x"]
    stage_norm = p.renorm == 2
    xi5 = vjp_normalize(xs[4], lam_out) if p.renorm >= 1 else lam_out
    lam = xi5.copy()
    kbar = [dt * b * xi5 for b in RK4_B]
    hbar = np.zeros(3)
    for s in (3, 2, 1, 0):
        ybar, mu = vjp_rhs(grid, p, ys[s], Hs[s], kbar[s], spec, pshape)
        if p.has(field.TERM_ZEEMAN):
            hbar += mu.reshape(3, -1).sum(axis=1)
        if s == 0:
            lam = lam + ybar
        else:
            xi = vjp_normalize(xs[s], ybar) if stage_norm else ybar
            lam = lam + xi
            kbar[s - 1] = kbar[s - 1] + RK4_C[s] * dt * xi
    return lam, hbar


def masked_mean_mz(mask, m):
    """Loss L = sum_i mask_i m_z,i / sum_i mask_i."""
    return float(np.sum(mask * m[2]) / np.sum(mask))


def masked_mean_mz_grad(mask, m):
    g = np.zeros_like(m, dtype=np.float64)
    g[2] = mask / np.sum(mask)
    return g


def rollout(grid, p, m0, dt, nsteps, spec=None, pshape=None):
    m = np.asarray(m0, dtype=np.float64)
    for _ in range(nsteps):
        m = llg.rk4_step(grid, p, m, dt, spec, pshape)
    return m


def rollout_grad(grid, p, m0, dt, nsteps, ckpt, mask, spec=None, pshape=None):
    """Loss, dL/dm0 and dL/dHbias for L = masked mean of m_z after nsteps,
    with m stored every `ckpt` steps and each segment recomputed."""
    ckpt = max(1, min(ckpt, nsteps)) if nsteps > 0 else 1
    saved = {0: np.asarray(m0, dtype=np.float64)}
    m = saved[0]
    for n in range(nsteps):
        m = llg.rk4_step(grid, p, m, dt, spec, pshape)
        if (n + 1) % ckpt == 0 and n + 1 < nsteps:
            saved[n + 1] = m
    loss = masked_mean_mz(mask, m)
    lam = masked_mean_mz_grad(mask, m)
    hbar = np.zeros(3)
    starts = sorted(saved)
    for si in reversed(range(len(starts))):
        s0 = starts[si]
        s1 = starts[si + 1] if si + 1 < len(starts) else nsteps
        states = [saved[s0]]
        for _ in range(s0, s1 - 1):
            states.append(llg.rk4_step(grid, p, states[-1], dt, spec, pshape))
        for mn in reversed(states):
            lam, hb = rk4_step_vjp(grid, p, mn, dt, lam, spec, pshape)
            hbar += hb
    return loss, lam, hbar
