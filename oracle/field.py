"""Effective field H_eff(m) on the cell-centred grid (FP64 oracle, test infrastructure only).

Eq. (2): H_eff = H_bias + H_demag + H_ani + H_exch + H_DMI, with m = M/Ms a
(3, nz, ny, nx) array, x fastest.

* Exchange, Eq. (7) with uniform A: H = (2A/(mu0 Ms)) lap(m), second-order
  central differences (Section II-B).
* Interfacial DMI, Eq. (9): H = -(2D/(mu0 Ms)) [(div m) e_z - grad m_z], i.e.
  H_x = c dm_z/dx, H_y = c dm_z/dy, H_z = -c (dm_x/dx + dm_y/dy), c = 2D/(mu0 Ms),
  central differences.
* Boundary condition (Section II-B, Eq. (10)): zero-flux Neumann without DMI;
  with DMI, dm/dn = -(D/2A)(e_z x n) x m on a face with outward normal n.  It is
  imposed with one ghost cell per face, m_ghost = m_b + h_n dm/dn, used by both
  the exchange and the DMI stencil.  On z faces e_z x e_z = 0, so the condition
  is plain Neumann there.
* Uniaxial anisotropy, Eq. (5): H = (2Ku/(mu0 Ms)) (m.eK) eK.
* Zeeman: the uniform bias field.
* Demagnetisation: oracle.demag.
"""
import numpy as np

from . import demag
from .params import TERM_DEMAG, TERM_EXCH, TERM_DMI, TERM_ANIS, TERM_ZEEMAN

EZ = np.array([0.0, 0.0, 1.0])


def _cross(a, b):
    """Cross product of (3, ...) arrays."""
    return np.stack([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def ghost_padded(grid, p, m):
    """m with one ghost layer on every face: shape (3, nz+2, ny+2, nx+2).

    Edge and corner ghosts are not used by the 7-point stencil and stay 0.
    """
    nz, ny, nx = grid.shape
    g = np.zeros((3, nz + 2, ny + 2, nx + 2))
    g[:, 1:-1, 1:-1, 1:-1] = m
    dmi = p.has(TERM_DMI) and p.D != 0.0
    kappa = -p.D / (2.0 * p.A) if dmi else 0.0

    def ghost(mb, normal, h):
        if not dmi:
            return mb.copy()
        axis = np.cross(EZ, normal)  # e_z x n
        ax = axis.reshape(3, *([1] * (mb.ndim - 1)))
        return mb + h * kappa * _cross(np.broadcast_to(ax, mb.shape), mb)

    g[:, 1:-1, 1:-1, 0] = ghost(m[:, :, :, 0], np.array([-1.0, 0, 0]), grid.dx)
    g[:, 1:-1, 1:-1, -1] = ghost(m[:, :, :, -1], np.array([1.0, 0, 0]), grid.dx)
    g[:, 1:-1, 0, 1:-1] = ghost(m[:, :, 0, :], np.array([0, -1.0, 0]), grid.dy)
    g[:, 1:-1, -1, 1:-1] = ghost(m[:, :, -1, :], np.array([0, 1.0, 0]), grid.dy)
    g[:, 0, 1:-1, 1:-1] = m[:, 0]
    g[:, -1, 1:-1, 1:-1] = m[:, -1]
    return g


def _neighbours(g):
    c = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    xp = g[:, 1:-1, 1:-1, 2:]
    xm = g[:, 1:-1, 1:-1, :-2]
    yp = g[:, 1:-1, 2:, 1:-1]
    ym = g[:, 1:-1, :-2, 1:-1]
    zp = g[:, 2:, 1:-1, 1:-1]
    zm = g[:, :-2, 1:-1, 1:-1]
    return g[c], xp, xm, yp, ym, zp, zm


def exchange(grid, p, m, g=None):
    g = ghost_padded(grid, p, m) if g is None else g
    c, xp, xm, yp, ym, zp, zm = _neighbours(g)
    lap = (xp - 2 * c + xm) / grid.dx ** 2 + (yp - 2 * c + ym) / grid.dy ** 2 + (zp - 2 * c + zm) / grid.dz ** 2
    return (2.0 * p.A / (p.mu0 * p.Ms)) * lap


def dmi(grid, p, m, g=None):
    g = ghost_padded(grid, p, m) if g is None else g
    c, xp, xm, yp, ym, zp, zm = _neighbours(g)
    ddx = (xp - xm) / (2 * grid.dx)
    ddy = (yp - ym) / (2 * grid.dy)
    k = 2.0 * p.D / (p.mu0 * p.Ms)
    H = np.empty_like(c)
    H[0] = k * ddx[2]
    H[1] = k * ddy[2]
    H[2] = -k * (ddx[0] + ddy[1])
    return H


def anisotropy(p, m):
    e = np.asarray(p.eK, dtype=np.float64)
    proj = np.tensordot(e, m, axes=(0, 0))
    return (2.0 * p.Ku / (p.mu0 * p.Ms)) * e.reshape(3, 1, 1, 1) * proj[None]


def check_params(p):
    if p.has(TERM_DMI) and p.D != 0.0:
        if not p.has(TERM_EXCH) or p.A <= 0.0:
            raise ValueError("DMI boundary condition needs exchange with A > 0")


# ---- geometry masks and space-dependent Ms (NEXT row f3) -------------------------
# Ms(r) = Ms s(r) with s = p.ms_profile; s = 0 marks cells outside the magnet.
# The demagnetising field is that of M = Ms(r) m (Eq. (3)); the local terms of
# a cell use its own Ms in their prefactors (Eqs. (5), (7), (9)); the surface of
# the magnet is a boundary like the faces of the grid: a neighbour outside the
# magnet is replaced by the ghost of Eq. (10) built from the cell itself.  Cells
# outside the magnet carry no field.

def _masked_neighbours(grid, p, m, s):
    """For each of the six directions, the neighbour values seen by every cell:
    the neighbouring cell if it lies in the grid and in the magnet, else the
    ghost m + h dm/dn of the boundary condition."""
    dmi_on = p.has(TERM_DMI) and p.D != 0.0
    kappa = -p.D / (2.0 * p.A) if dmi_on else 0.0
    inside = s > 0
    out = {}
    for name, axis, sign, h in (("xp", 3, 1, grid.dx), ("xm", 3, -1, grid.dx), ("yp", 2, 1, grid.dy),
                                ("ym", 2, -1, grid.dy), ("zp", 1, 1, grid.dz), ("zm", 1, -1, grid.dz)):
        nb = np.zeros_like(m)
        ok = np.zeros(m.shape[1:], dtype=bool)
        src = [slice(None)] * 4
        dst = [slice(None)] * 4
        if sign > 0:
            src[axis], dst[axis] = slice(1, None), slice(0, -1)
        else:
            src[axis], dst[axis] = slice(0, -1), slice(1, None)
        nb[tuple(dst)] = m[tuple(src)]
        ok[tuple(dst[1:])] = inside[tuple(src[1:])]
        normal = np.zeros(3)
        normal[3 - axis] = float(sign)          # axis 3 -> x, 2 -> y, 1 -> z
        if dmi_on:
            ax = np.cross(EZ, normal).reshape(3, 1, 1, 1)
            ghost = m + h * kappa * _cross(np.broadcast_to(ax, m.shape), m)
        else:
            ghost = m
        out[name] = np.where(ok[None], nb, ghost)
    return out


def heff_parts_masked(grid, p, m, spec=None, pshape=None):
    s = np.asarray(p.ms_profile, dtype=np.float64)
    if s.shape != tuple(grid.shape) or np.any(s < 0):
        raise ValueError("ms_profile must be a non-negative (nz, ny, nx) array")
    inside = s > 0
    inv = np.where(inside, 1.0 / np.where(inside, s, 1.0), 0.0)      # 1/s inside, 0 outside
    parts = {}
    if p.has(TERM_DEMAG):
        parts["demag"] = demag.demag_fft(grid, p.Ms * s, m, spec=spec, pshape=pshape) * inside[None]
    if p.has(TERM_EXCH) or p.has(TERM_DMI):
        nb = _masked_neighbours(grid, p, m, s)
        if p.has(TERM_EXCH):
            lap = ((nb["xp"] - 2 * m + nb["xm"]) / grid.dx ** 2 + (nb["yp"] - 2 * m + nb["ym"]) / grid.dy ** 2 +
                   (nb["zp"] - 2 * m + nb["zm"]) / grid.dz ** 2)
            parts["exch"] = (2.0 * p.A / (p.mu0 * p.Ms)) * inv[None] * lap
        if p.has(TERM_DMI):
            ddx = (nb["xp"] - nb["xm"]) / (2 * grid.dx)
            ddy = (nb["yp"] - nb["ym"]) / (2 * grid.dy)
            k = (2.0 * p.D / (p.mu0 * p.Ms)) * inv
            parts["dmi"] = np.stack([k * ddx[2], k * ddy[2], -k * (ddx[0] + ddy[1])])
    if p.has(TERM_ANIS):
        parts["anis"] = anisotropy(p, m) * inv[None]
    if p.has(TERM_ZEEMAN):
        parts["zeeman"] = np.asarray(p.Hbias, np.float64).reshape(3, 1, 1, 1) * inside[None]
    return parts


def heff_parts(grid, p, m, spec=None, pshape=None):
    """Dictionary of the enabled field terms (A/m)."""
    check_params(p)
    m = np.asarray(m, dtype=np.float64)
    if getattr(p, "ms_profile", None) is not None:
        return heff_parts_masked(grid, p, m, spec, pshape)
    parts = {}
    if p.has(TERM_DEMAG):
        parts["demag"] = demag.demag_fft(grid, p.Ms, m, spec=spec, pshape=pshape)
    if p.has(TERM_EXCH) or p.has(TERM_DMI):
        g = ghost_padded(grid, p, m)
        if p.has(TERM_EXCH):
            parts["exch"] = exchange(grid, p, m, g)
        if p.has(TERM_DMI):
            parts["dmi"] = dmi(grid, p, m, g)
    if p.has(TERM_ANIS):
        parts["anis"] = anisotropy(p, m)
    if p.has(TERM_ZEEMAN):
        parts["zeeman"] = np.broadcast_to(np.asarray(p.Hbias, np.float64).reshape(3, 1, 1, 1), m.shape).copy()
    return parts


def heff(grid, p, m, spec=None, pshape=None):
    """Eq. (2): sum of the enabled terms."""
    parts = heff_parts(grid, p, m, spec, pshape)
    H = np.zeros(np.shape(m))
    for v in parts.values():
        H = H + v
    return H


def linear_part(grid, p, v, spec=None, pshape=None):
    """K v: H_eff of v with the bias field left out (the field is affine in m,
    H_eff(m) = K m + H_bias, and K is linear because the ghost rule is)."""
    from dataclasses import replace
    q = replace(p, terms=p.terms & ~TERM_ZEEMAN)
    return heff(grid, q, v, spec, pshape)
