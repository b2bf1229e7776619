"""Demagnetising tensor of two rectangular cells (FP64 oracle, test infrastructure only).

Definition (Section II-B and Eq. (3) of the paper, with the sign convention
H = -N M; the paper's N absorbs that sign): for two dx*dy*dz cells whose
centres differ by R,

    N_ab(R) = -1/(4 pi V) * int_target int_source d_a d_b (1/|x-y|) dy dx,

i.e. minus the target-cell average of the field of a uniformly magnetised
source cell.  The paper cites the extended-grid method of Nakatani et al. and
Hayashi et al. but prints no formula; the cell-averaged (Newell-Williams-Dunlop
1993) tensor is used.

Two evaluations, chosen per offset by r = |R| / max(dx, dy, dz):

* near (r < R_NEAR): Newell's closed forms -- a 27-point product of the
  (-1, 2, -1) second difference along each axis, applied to the auxiliary
  functions f (diagonal components) or g (off-diagonal components), divided
  by 4 pi V.  Exact, but the difference cancels catastrophically as r grows.
* far (r >= R_NEAR): the same double integral written as an expectation,
  N(R) = -(V/4pi) E_v[K(R + v)],  K_ab(r) = d_a d_b (1/r) = (3 r_a r_b - r^2 delta_ab)/r^5,
  where v is the difference of two independent uniform points of a cell, so
  each v_i has the triangle density (d_i - |v_i|)/d_i^2 on [-d_i, d_i].  The
  expectation is taken with Gauss-Legendre on each half of each triangle; the
  number of nodes q per half falls with distance (QUAD_RULE).

Component order everywhere: xx, yy, zz, xy, xz, yz.
"""
import math
import numpy as np

R_NEAR = 6.0
# (upper bound on r, Gauss-Legendre nodes per triangle half)
QUAD_RULE = ((12.0, 6), (40.0, 5), (150.0, 4), (2000.0, 3), (math.inf, 2))

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")
# parity of each component along (x, y, z): +1 even, -1 odd
PARITY = {
    "xx": (1, 1, 1), "yy": (1, 1, 1), "zz": (1, 1, 1),
    "xy": (-1, -1, 1), "xz": (-1, 1, -1), "yz": (1, -1, -1),
}


def newell_f(x, y, z):
    """Newell's auxiliary function for N_xx (vectorised, FP64).

    Terms whose logarithm/arctangent argument degenerates are multiplied by a
    factor that vanishes faster, so they are set to their limit 0.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = (2.0 * x2 - y2 - z2) * R / 6.0
    with np.errstate(divide="ignore", invalid="ignore"):
        s = x2 + z2
        out = out + np.where(s > 0, 0.5 * y * (z2 - x2) * np.arcsinh(y / np.sqrt(s)), 0.0)
        s = x2 + y2
        out = out + np.where(s > 0, 0.5 * z * (y2 - x2) * np.arcsinh(z / np.sqrt(s)), 0.0)
        out = out + np.where((x != 0) & (R > 0), -x * y * z * np.arctan(y * z / (x * R)), 0.0)
    return out


def newell_g(x, y, z):
    """Newell's auxiliary function for N_xy (vectorised, FP64)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = -x * y * R / 3.0
    with np.errstate(divide="ignore", invalid="ignore"):
        s = x2 + y2
        out = out + np.where(s > 0, x * y * z * np.arcsinh(z / np.sqrt(s)), 0.0)
        s = y2 + z2
        out = out + np.where(s > 0, y / 6.0 * (3.0 * z2 - y2) * np.arcsinh(x / np.sqrt(s)), 0.0)
        s = x2 + z2
        out = out + np.where(s > 0, x / 6.0 * (3.0 * z2 - x2) * np.arcsinh(y / np.sqrt(s)), 0.0)
        out = out + np.where(z != 0, -z2 * z / 6.0 * np.arctan(x * y / (z * R)), 0.0)
        out = out + np.where(y != 0, -z * y2 / 2.0 * np.arctan(x * z / (y * R)), 0.0)
        out = out + np.where(x != 0, -z * x2 / 2.0 * np.arctan(y * z / (x * R)), 0.0)
    return out


_W3 = (-1.0, 2.0, -1.0)


def _second_difference(fn, X, Y, Z, a, b, c):
    """Sum over i,j,k in {-1,0,1} of w_i w_j w_k fn(X+i a, Y+j b, Z+k c) / (4 pi a b c)."""
    acc = 0.0
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                w = _W3[i + 1] * _W3[j + 1] * _W3[k + 1]
                acc = acc + w * fn(X + i * a, Y + j * b, Z + k * c)
    return acc / (4.0 * math.pi * a * b * c)


def near_tensor(X, Y, Z, dx, dy, dz):
    """All six components from Newell's closed forms (any offset, exact math)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    nxx = _second_difference(newell_f, X, Y, Z, dx, dy, dz)
    nyy = _second_difference(newell_f, Y, X, Z, dy, dx, dz)
    nzz = _second_difference(newell_f, Z, Y, X, dz, dy, dx)
    nxy = _second_difference(newell_g, X, Y, Z, dx, dy, dz)
    nxz = _second_difference(newell_g, X, Z, Y, dx, dz, dy)
    nyz = _second_difference(newell_g, Y, Z, X, dy, dz, dx)
    return np.stack(np.broadcast_arrays(nxx, nyy, nzz, nxy, nxz, nyz))


def triangle_nodes(d, q):
    """Nodes and weights for E[h(v)], v with density (d-|v|)/d^2 on [-d, d].

    Gauss-Legendre with q nodes on each half; the linear density is folded
    into the weights.  Weights sum to 1.
    """
    t, w = np.polynomial.legendre.leggauss(q)
    v = 0.5 * d * (t + 1.0)
    wv = w * 0.5 * d * (d - v) / (d * d)
    return np.concatenate([-v[::-1], v]), np.concatenate([wv[::-1], wv])


def far_tensor(X, Y, Z, dx, dy, dz, q):
    """N(R) = -(V/4pi) E_v[K(R+v)] with q Gauss-Legendre nodes per triangle half.

    Valid only when the two cells do not overlap (|R| well above the cell
    size); used for r >= R_NEAR.
    """
    X = np.atleast_1d(np.asarray(X, dtype=np.float64)).ravel()
    Y = np.atleast_1d(np.asarray(Y, dtype=np.float64)).ravel()
    Z = np.atleast_1d(np.asarray(Z, dtype=np.float64)).ravel()
    vx, wx = triangle_nodes(dx, q)
    vy, wy = triangle_nodes(dy, q)
    vz, wz = triangle_nodes(dz, q)
    W = (wx[:, None, None] * wy[None, :, None] * wz[None, None, :]).ravel()
    VX = np.broadcast_to(vx[:, None, None], (vx.size, vy.size, vz.size)).ravel()
    VY = np.broadcast_to(vy[None, :, None], (vx.size, vy.size, vz.size)).ravel()
    VZ = np.broadcast_to(vz[None, None, :], (vx.size, vy.size, vz.size)).ravel()
    scale = -(dx * dy * dz) / (4.0 * math.pi)
    out = np.empty((6, X.size))
    chunk = max(1, 4_000_000 // W.size)
    for s in range(0, X.size, chunk):
        x = X[s:s + chunk, None] + VX[None, :]
        y = Y[s:s + chunk, None] + VY[None, :]
        z = Z[s:s + chunk, None] + VZ[None, :]
        r2 = x * x + y * y + z * z
        inv5 = 1.0 / (r2 * r2 * np.sqrt(r2))
        out[0, s:s + chunk] = ((3.0 * x * x - r2) * inv5) @ W
        out[1, s:s + chunk] = ((3.0 * y * y - r2) * inv5) @ W
        out[2, s:s + chunk] = ((3.0 * z * z - r2) * inv5) @ W
        out[3, s:s + chunk] = (3.0 * x * y * inv5) @ W
        out[4, s:s + chunk] = (3.0 * x * z * inv5) @ W
        out[5, s:s + chunk] = (3.0 * y * z * inv5) @ W
    return scale * out


def quad_order(r):
    """Gauss-Legendre nodes per triangle half for normalised distance r >= R_NEAR."""
    for bound, q in QUAD_RULE:
        if r < bound:
            return q
    return QUAD_RULE[-1][1]


def tensor(X, Y, Z, dx, dy, dz):
    """N_ab at arbitrary offsets (arrays broadcast together); returns (6, ...)."""
    X, Y, Z = np.broadcast_arrays(np.asarray(X, np.float64), np.asarray(Y, np.float64),
                                  np.asarray(Z, np.float64))
    shape = X.shape
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    r = np.sqrt(X * X + Y * Y + Z * Z) / max(dx, dy, dz)
    out = np.empty((6, X.size))
    near = r < R_NEAR
    if near.any():
        out[:, near] = near_tensor(X[near], Y[near], Z[near], dx, dy, dz)
    lo = R_NEAR
    for bound, q in QUAD_RULE:
        sel = (r >= lo) & (r < bound)
        if sel.any():
            out[:, sel] = far_tensor(X[sel], Y[sel], Z[sel], dx, dy, dz, q)
        lo = bound
    return out.reshape((6,) + shape)


def octant(grid):
    """Real-space tensor at all non-negative cell offsets: shape (6, nz, ny, nx).

    Entry [c, k, j, i] is component c at R = (i dx, j dy, k dz).
    """
    k, j, i = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx), indexing="ij")
    return tensor(i * grid.dx, j * grid.dy, k * grid.dz, grid.dx, grid.dy, grid.dz)


def padded_shape(grid):
    """Extended grid of twice the problem size along each axis (Section II-B)."""
    return (2 * grid.nz, 2 * grid.ny, 2 * grid.nx)


def padded(grid, pshape=None, oct_=None):
    """Tensor on the extended grid, offsets placed with wrap-around.

    Offset (I, J, K) with |I| < nx etc. goes to index (I mod Px, ...); every
    other entry of the extended grid (offsets the convolution never reaches,
    such as +-nx when Px = 2 nx) is zero.  Negative offsets are filled from the
    octant with each component's parity.
    """
    Pz, Py, Px = pshape if pshape is not None else padded_shape(grid)
    assert Px >= 2 * grid.nx - 1 and Py >= 2 * grid.ny - 1 and Pz >= 2 * grid.nz - 1
    oc = octant(grid) if oct_ is None else oct_
    out = np.zeros((6, Pz, Py, Px))
    nz, ny, nx = grid.nz, grid.ny, grid.nx
    for c, name in enumerate(COMPONENTS):
        px, py, pz = PARITY[name]
        for sz in (1, -1):
            for sy in (1, -1):
                for sx in (1, -1):
                    sign = (px if sx < 0 else 1) * (py if sy < 0 else 1) * (pz if sz < 0 else 1)
                    iz = (sz * np.arange(nz)) % Pz
                    iy = (sy * np.arange(ny)) % Py
                    ix = (sx * np.arange(nx)) % Px
                    out[c][np.ix_(iz, iy, ix)] = sign * oc[c]
    return out


def spectrum(grid, pshape=None):
    """Real spectrum of each component on the extended grid: (6, Pz, Py, Px//2+1).

    Each component is even or odd along every axis and odd along an even
    number of axes, so its DFT is real; the imaginary part is checked to
    vanish to rounding.
    """
    import scipy.fft as sfft
    full = padded(grid, pshape)
    spec = sfft.rfftn(full, axes=(1, 2, 3), workers=_workers())
    scale = np.abs(spec.real).max()
    assert np.abs(spec.imag).max() <= 1e-12 * max(scale, 1e-300) + 1e-300, "tensor spectrum not real"
    return spec.real.copy()


def _workers():
    import os
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
