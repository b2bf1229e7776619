"""Demagnetising field by zero-padded FFT convolution, and the direct sum it equals.

Section II-B of the paper: M is zero-padded to an extended grid of twice the
problem size along each axis and circularly convolved with the real-space
tensor placed on that grid, which equals the open-boundary linear
convolution of Eq. (3):

    H_demag(r_i) = -Ms * sum_j N(r_i - r_j) m_j          (H = -N M).

`demag_direct` is that sum written out (O(N^2), tiny grids only);
`demag_fft` is the extended-grid FFT route.  Test infrastructure only.
"""
import numpy as np
import scipy.fft as sfft

from . import newell


def demag_direct(grid, Ms, m):
    """O(N^2) sum over all source cells; the tensor is evaluated at every
    signed offset directly (no parity folding).  Ms may be a scalar or a
    per-cell array (nz, ny, nx): the source is M = Ms m."""
    nz, ny, nx = grid.shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)  # (N, 3) cell indices
    n = pos.shape[0]
    off = pos[:, None, :] - pos[None, :, :]                      # target - source
    T = newell.tensor(off[..., 0] * grid.dx, off[..., 1] * grid.dy, off[..., 2] * grid.dz,
                      grid.dx, grid.dy, grid.dz)                  # (6, N, N)
    full = np.empty((3, 3, n, n))
    full[0, 0], full[1, 1], full[2, 2] = T[0], T[1], T[2]
    full[0, 1] = full[1, 0] = T[3]
    full[0, 2] = full[2, 0] = T[4]
    full[1, 2] = full[2, 1] = T[5]
    Mv = (np.asarray(Ms, dtype=np.float64) * m).reshape(3, n)
    H = -np.einsum("abij,bj->ai", full, Mv)
    return H.reshape(m.shape)


def demag_fft(grid, Ms, m, spec=None, pshape=None):
    """Extended-grid FFT convolution.  spec: output of newell.spectrum.  Ms
    may be a scalar or a per-cell array (nz, ny, nx)."""
    pz, py, px = pshape if pshape is not None else newell.padded_shape(grid)
    if spec is None:
        spec = newell.spectrum(grid, (pz, py, px))
    nz, ny, nx = grid.shape
    w = newell._workers()
    Mhat = []
    for b in range(3):
        buf = np.zeros((pz, py, px))
        buf[:nz, :ny, :nx] = Ms * m[b]
        Mhat.append(sfft.rfftn(buf, workers=w))
    xx, yy, zz, xy, xz, yz = spec
    Hhat = (
        -(xx * Mhat[0] + xy * Mhat[1] + xz * Mhat[2]),
        -(xy * Mhat[0] + yy * Mhat[1] + yz * Mhat[2]),
        -(xz * Mhat[0] + yz * Mhat[1] + zz * Mhat[2]),
    )
    H = np.empty_like(m, dtype=np.float64)
    for a in range(3):
        H[a] = sfft.irfftn(Hhat[a], s=(pz, py, px), workers=w)[:nz, :ny, :nx]
    return H
