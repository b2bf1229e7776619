"""Seeded synthetic workloads for the LLG hot path.

This module only generates inputs: grid sizes, material constants and seeded
random fields.  It holds none of the method's arithmetic and imports neither
the oracle nor the GPU package; both sides take their inputs from here.

Workloads (the paper's benchmark geometries and materials, Section III; the
random states stand in for the standard-problem initial conditions):

  film     128x32x1 cells of 3.90625x3.90625x3 nm (the Standard Problem 4
           film size), permalloy Ms 8e5, A 1.3e-11, alpha 0.02, 25 mT along x
  dmi      256x256x16 cubic 2 nm cells, Ms 1.1e6, A 1.6e-11, Ku 1e6 along z,
           D 3e-3, alpha 0.3, 1000 RK4 steps of 1e-13 s, unsmoothed start
  demag    512x512x32 cells of 2.5 nm, Ms 8e5, A 1.3e-11, alpha 0.5,
           200 RK4 steps of 1e-13 s (the throughput headline)
  adjoint  256x256x8 cells of 2 nm, Ms 1e6, A 1.6e-11, Ku 8e5 along z,
           D 2.5e-3, alpha 0.1, 100 steps of 5e-14 s, loss = masked mean m_z,
           checkpoint every 10 steps
  large    1024x1024x64 cells of 3 nm, Ms 8e5, A 1.3e-11, alpha 0.02,
           10 mT along a seeded random direction, 50 steps, checkpoint 10,
           the adjoint workload's loss form with its own mask (seed 2005)
  sp4_fine the Standard Problem 4 film (500 x 125 x 3.125 nm) at 0.78125 nm
           cells, 640x160x4, permalloy, field 1 (mu0 H = (-24.6, 4.3, 0) mT),
           demag + exchange + Zeeman: the integrator comparison of the paper
           (RK4 at dt 2.5e-14 s against multirate at 1.25e-13 s with fast
           steps of 1.25e-14 s over one 1.25e-13 s interval), starting from
           a smooth S-like texture (no seed)

Magnetisation starts are random unit vectors (normalised N(0,1)^3), optionally
smoothed by damped neighbour-averaging passes and renormalised, generated in
float64 and rounded once to float32; both sides then start from the same
float32 values.  Field values quoted in mT are B = mu0 H, so H = B / mu0.
"""
import math
from dataclasses import dataclass, field

import numpy as np

MU0 = 4.0e-7 * math.pi
GAMMA = -1.759e11

TERM_DEMAG, TERM_EXCH, TERM_DMI, TERM_ANIS, TERM_ZEEMAN = 1, 2, 4, 8, 16


@dataclass
class Workload:
    name: str
    n: tuple            # (nx, ny, nz)
    d: tuple            # (dx, dy, dz) in metres
    Ms: float
    A: float
    alpha: float
    terms: int
    D: float = 0.0
    Ku: float = 0.0
    eK: tuple = (0.0, 0.0, 1.0)
    Hbias: tuple = (0.0, 0.0, 0.0)
    steps: int = 1
    dt: float = 1e-13
    seed: int = 0
    smooth: int = 3
    ckpt: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def ncell(self):
        return self.n[0] * self.n[1] * self.n[2]

    def material(self):
        """Plain dict of material/physics constants (SI units)."""
        return dict(Ms=self.Ms, A=self.A, D=self.D, Ku=self.Ku, eK=tuple(self.eK),
                    Hbias=tuple(self.Hbias), alpha=self.alpha, gamma=GAMMA, mu0=MU0,
                    terms=self.terms, renorm=2)


def _direction(seed):
    v = np.random.default_rng(seed).standard_normal(3)
    return tuple(float(x) for x in v / np.linalg.norm(v))


def _workloads():
    h25 = 0.025 / MU0
    h10 = 0.010 / MU0
    d10 = _direction(4005)
    return {
        "film": Workload("film", (128, 32, 1), (3.90625e-9, 3.90625e-9, 3e-9), 8.0e5, 1.3e-11, 0.02,
                         TERM_DEMAG | TERM_EXCH | TERM_ZEEMAN, Hbias=(h25, 0.0, 0.0),
                         steps=1, dt=1e-13, seed=1001, smooth=3),
        "dmi": Workload("dmi", (256, 256, 16), (2e-9, 2e-9, 2e-9), 1.1e6, 1.6e-11, 0.3,
                        TERM_DEMAG | TERM_EXCH | TERM_DMI | TERM_ANIS, D=3e-3, Ku=1e6,
                        steps=1000, dt=1e-13, seed=1002, smooth=0),
        "demag": Workload("demag", (512, 512, 32), (2.5e-9, 2.5e-9, 2.5e-9), 8.0e5, 1.3e-11, 0.5,
                          TERM_DEMAG | TERM_EXCH, steps=200, dt=1e-13, seed=1003, smooth=3,
                          ckpt=10),
        "adjoint": Workload("adjoint", (256, 256, 8), (2e-9, 2e-9, 2e-9), 1.0e6, 1.6e-11, 0.1,
                            TERM_DEMAG | TERM_EXCH | TERM_DMI | TERM_ANIS | TERM_ZEEMAN,
                            D=2.5e-3, Ku=8e5, steps=100, dt=5e-14, seed=1004, smooth=3, ckpt=10,
                            extra=dict(mask_seed=2004, fd_seeds=list(range(3000, 3064)))),
        "large": Workload("large", (1024, 1024, 64), (3e-9, 3e-9, 3e-9), 8.0e5, 1.3e-11, 0.02,
                          TERM_DEMAG | TERM_EXCH | TERM_ZEEMAN,
                          Hbias=tuple(h10 * c for c in d10), steps=50, dt=1e-13, seed=1005,
                          smooth=3, ckpt=10, extra=dict(mask_seed=2005)),
        "sp4_fine": Workload("sp4_fine", (640, 160, 4), (0.78125e-9, 0.78125e-9, 0.78125e-9), 8.0e5, 1.3e-11,
                             0.02, TERM_DEMAG | TERM_EXCH | TERM_ZEEMAN,
                             Hbias=(-0.0246 / MU0, 0.0043 / MU0, 0.0), steps=5, dt=2.5e-14, seed=1006,
                             smooth=0, extra=dict(dt_mri=1.25e-13, dt_fast=1.25e-14, interval=1.25e-13,
                                                  texture="s_like")),
    }


WORKLOADS = _workloads()


def random_unit_field(n, seed, smooth=0):
    """Seeded unit-vector field of shape (3, nz, ny, nx), float64 before rounding.

    Gaussian triples normalised per cell, then `smooth` damped passes
    m_i <- (m_i + sum of in-grid face neighbours) / (1 + count), renormalised
    after the passes.
    """
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, nz, ny, nx))
    v /= np.sqrt(np.sum(v * v, axis=0))[None]
    for _ in range(smooth):
        acc = v.copy()
        cnt = np.ones((nz, ny, nx))
        for axis in (1, 2, 3):
            size = v.shape[axis]
            if size < 2:
                continue
            lo = [slice(None)] * 4
            hi = [slice(None)] * 4
            lo[axis] = slice(0, size - 1)
            hi[axis] = slice(1, size)
            acc[tuple(lo)] += v[tuple(hi)]
            acc[tuple(hi)] += v[tuple(lo)]
            cl = [slice(None)] * 3
            ch = [slice(None)] * 3
            cl[axis - 1] = slice(0, size - 1)
            ch[axis - 1] = slice(1, size)
            cnt[tuple(cl)] += 1
            cnt[tuple(ch)] += 1
        v = acc / cnt[None]
    if smooth:
        v /= np.sqrt(np.sum(v * v, axis=0))[None]
    return v


def s_like_texture(n):
    """Smooth in-plane texture standing in for the relaxed S-state of the
    Standard Problem 4 film: m = (cos t cos p, cos t sin p, sin t) with
    p = 0.6 cos(pi u) sin(pi (v - 1/2)) and t = 0.08 sin(pi u), u, v the cell
    centres scaled to [0, 1] along x and y (the same in every layer)."""
    nx, ny, nz = n
    u = (np.arange(nx) + 0.5) / nx
    v = (np.arange(ny) + 0.5) / ny
    U, V = np.meshgrid(u, v, indexing="xy")             # (ny, nx)
    ph = 0.6 * np.cos(np.pi * U) * np.sin(np.pi * (V - 0.5))
    th = 0.08 * np.sin(np.pi * U)
    m = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), np.sin(th)])
    return np.broadcast_to(m[:, None], (3, nz, ny, nx)).copy()


def initial_state(w, dtype=np.float32):
    """Initial magnetisation of a workload, rounded once to `dtype`."""
    if w.extra.get("texture") == "s_like":
        return s_like_texture(w.n).astype(dtype)
    return random_unit_field(w.n, w.seed, w.smooth).astype(dtype)


def random_vector_field(n, seed, dtype=np.float64):
    """Plain N(0,1) vector field (3, nz, ny, nx), e.g. for cotangents."""
    nx, ny, nz = n
    return np.random.default_rng(seed).standard_normal((3, nz, ny, nx)).astype(dtype)


def bernoulli_mask(n, seed, p=0.5):
    """Seeded 0/1 mask of shape (nz, ny, nx); at least one cell is set."""
    nx, ny, nz = n
    mask = (np.random.default_rng(seed).random((nz, ny, nx)) < p).astype(np.float64)
    if mask.sum() == 0:
        mask.flat[0] = 1.0
    return mask


def tangent_direction(m, seed):
    """Seeded direction field tangent to m in every cell, scaled to unit RMS
    per cell (sum of |v_i|^2 equals the cell count)."""
    v = np.random.default_rng(seed).standard_normal(m.shape)
    v -= m * np.sum(m * v, axis=0)[None]
    ncell = m[0].size
    v *= math.sqrt(ncell / float(np.sum(v * v)))
    return v


def small_grid(n, d=(2e-9, 2e-9, 2e-9)):
    """Helper for tests: a workload-like tuple of a small grid."""
    return tuple(n), tuple(d)
