"""Writes the stored expected values of the full-size workload tests.

Calls only the FP64 oracle (oracle/) and the seeded input generators
(workloads/); nothing here touches the GPU library.  Run from the repository
root:

    python tests/golden/make_workload_golden.py demag512   # ~5 min on 8 cores
    python tests/golden/make_workload_golden.py adjoint256 # ~15 min
    python tests/golden/make_workload_golden.py film dmi256 adjoint256_cells  # ~2 min

demag512_sampled.npz -- the 512 x 512 x 32 demag workload (Section II-B
    convolution + exchange): the oracle's H_eff (Eq. (2)) and the state after
    one RK4 step (the workload's dt) at 4096 seeded cells plus the box's
    corners and face centres, and max_i |H_i| over every cell (the
    denominator of the normwise error).
film_sampled.npz, dmi256_sampled.npz, adjoint256_sampled.npz -- the same for
    the 128 x 32 x 1 film (every cell), the 256 x 256 x 16 DMI workload and the
    256 x 256 x 8 adjoint workload.
adjoint256_grad.npz -- the 256 x 256 x 8 adjoint workload: loss L = masked
    mean of m_z after 100 RK4 steps of 5e-14 s (mask seed 2004), the oracle's
    checkpointed reverse sweep (checkpoint every 10 steps): dL/dm0 projected on
    the 64 seeded tangent directions (seeds 3000-3063) and dL/dH_bias.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import adjoint as oadj  # noqa: E402
from oracle import field as ofield  # noqa: E402
from oracle import llg as ollg  # noqa: E402
from oracle import newell as onewell  # noqa: E402
from oracle.params import Grid, Params  # noqa: E402
from workloads import WORKLOADS, bernoulli_mask, initial_state, tangent_direction  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLE_SEED = 7001
NSAMPLE = 4096


def _params(mat):
    return Params(**{k: mat[k] for k in ("Ms", "A", "D", "Ku", "eK", "Hbias", "alpha", "terms", "renorm")})


def sample_cells(n, seed=SAMPLE_SEED, k=NSAMPLE):
    """Seeded distinct cells (x, y, z) plus the 8 corners and the 6 face centres."""
    nx, ny, nz = n
    flat = np.random.default_rng(seed).choice(nx * ny * nz, size=k, replace=False)
    z, rem = np.divmod(flat, nx * ny)
    y, x = np.divmod(rem, nx)
    pts = [tuple(v) for v in np.stack([x, y, z], 1)]
    for cx in (0, nx - 1):
        for cy in (0, ny - 1):
            for cz in (0, nz - 1):
                pts.append((cx, cy, cz))
    for f in ((0, ny // 2, nz // 2), (nx - 1, ny // 2, nz // 2), (nx // 2, 0, nz // 2),
              (nx // 2, ny - 1, nz // 2), (nx // 2, ny // 2, 0), (nx // 2, ny // 2, nz - 1)):
        pts.append(f)
    out = []
    seen = set()
    for p in pts:
        if p not in seen:
            seen.add(p)
            out.append(p)
    return np.array(out, dtype=np.int64)


def sampled(wname, fname):
    w = WORKLOADS[wname]
    g = Grid(*w.n, *w.d)
    p = _params(w.material())
    t0 = time.time()
    spec = onewell.spectrum(g)
    print(f"spectrum {time.time() - t0:.1f} s", flush=True)
    m = initial_state(w).astype(np.float64)
    H = ofield.heff(g, p, m, spec)
    print(f"heff {time.time() - t0:.1f} s", flush=True)
    m1 = ollg.rk4_step(g, p, m, w.dt, spec)
    print(f"rk4 step {time.time() - t0:.1f} s", flush=True)
    cells = sample_cells(w.n, k=min(NSAMPLE, w.ncell))
    x, y, z = cells[:, 0], cells[:, 1], cells[:, 2]
    hmax = float(np.sqrt((H ** 2).sum(0)).max())
    np.savez_compressed(os.path.join(HERE, fname), cells=cells,
                        H=H[:, z, y, x].T.copy(), m1=m1[:, z, y, x].T.copy(), hmax=hmax,
                        dt=w.dt, seed=w.seed)
    print(f"wrote {fname}: {len(cells)} cells, hmax {hmax:.6e}", flush=True)


def adjoint256():
    w = WORKLOADS["adjoint"]
    g = Grid(*w.n, *w.d)
    p = _params(w.material())
    t0 = time.time()
    spec = onewell.spectrum(g)
    print(f"spectrum {time.time() - t0:.1f} s", flush=True)
    m0 = initial_state(w).astype(np.float64)
    mask = bernoulli_mask(w.n, w.extra["mask_seed"])
    loss, gm, gh = oadj.rollout_grad(g, p, m0, w.dt, w.steps, w.ckpt, mask, spec)
    print(f"gradient {time.time() - t0:.1f} s", flush=True)
    seeds = np.array(w.extra["fd_seeds"], dtype=np.int64)
    proj = np.array([float(np.sum(gm * tangent_direction(m0, int(s)))) for s in seeds])
    np.savez_compressed(os.path.join(HERE, "adjoint256_grad.npz"), loss=loss, proj=proj, seeds=seeds,
                        gHbias=np.asarray(gh, dtype=np.float64), gm_rms=float(np.sqrt(np.mean(gm ** 2))),
                        steps=w.steps, ckpt=w.ckpt, dt=w.dt)
    print(f"wrote adjoint256_grad.npz: loss {loss:.12e}, dL/dH_bias {gh}", flush=True)


if __name__ == "__main__":
    jobs = {"demag512": lambda: sampled("demag", "demag512_sampled.npz"),
            "film": lambda: sampled("film", "film_sampled.npz"),
            "dmi256": lambda: sampled("dmi", "dmi256_sampled.npz"),
            "adjoint256_cells": lambda: sampled("adjoint", "adjoint256_sampled.npz"),
            "adjoint256": adjoint256}
    for name in sys.argv[1:] or list(jobs):
        jobs[name]()
