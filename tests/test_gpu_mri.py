"""GPU parity of the multirate step (Section III-C: explicit-explicit MRI,
Knoth-Wolke on both scales, exchange torque as the fast partition) against
the FP64 oracle, through the C ABI.  Same normwise errors and bars as the RK4
parity tests: 1e-11 in double precision, 1e-5 in single precision per step."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import mri as omri  # noqa: E402
from oracle import newell as onewell  # noqa: E402
from oracle.params import Grid, Params  # noqa: E402
from workloads import random_unit_field  # noqa: E402

ALL = 31
CASES = {
    "tiny_all": ((7, 5, 3), (2e-9, 2.5e-9, 1.5e-9),
                 dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, eK=(0.0, 0.6, 0.8), alpha=0.1,
                      Hbias=(2e4, -1e4, 3e4), terms=ALL)),
    "ragged_dmi": ((37, 11, 5), (2e-9, 2e-9, 2e-9),
                   dict(Ms=1.1e6, A=1.6e-11, D=3e-3, Ku=1e6, eK=(0, 0, 1), alpha=0.3, terms=1 | 2 | 4 | 8)),
    "sp4_like": ((40, 10, 1), (3.125e-9, 3.125e-9, 3e-9),
                 dict(Ms=8e5, A=1.3e-11, alpha=0.02, Hbias=(-19576.0, 3422.0, 0.0), terms=1 | 2 | 16)),
    "line": ((33, 1, 1), (3e-9, 3e-9, 3e-9),
             dict(Ms=8e5, A=1.3e-11, D=1e-3, alpha=0.02, Hbias=(0, 0, 1e4), terms=ALL)),
    "no_demag": ((12, 9, 2), (2e-9, 2e-9, 1e-9),
                 dict(Ms=5.8e5, A=1.5e-11, D=3e-3, Ku=8e5, alpha=0.3, terms=2 | 4 | 8)),
    "tiles": ((96, 70, 9), (2e-9, 2e-9, 3e-9),
              dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, alpha=0.1, Hbias=(1e3, 2e3, -5e3), terms=ALL)),
}
_SPEC = {}


def _magx():
    from paper_2602_12242_amd import magx
    return magx


def _spec(name):
    if name not in _SPEC:
        n, d, _ = CASES[name]
        g = Grid(*n, *d)
        P = tuple(max(2, 1 << (2 * v - 1).bit_length()) for v in (n[2], n[1], n[0]))
        _SPEC[name] = (g, onewell.spectrum(g, P), P)
    return _SPEC[name]


def _err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.sqrt(((a - b) ** 2).sum(0)).max() / np.sqrt((b ** 2).sum(0)).max()


def _run(name, dtype, renorm, dt, dt_fast, nsteps, seed=801):
    magx = _magx()
    n, d, mat = CASES[name]
    g, spec, P = _spec(name)
    m0 = random_unit_field(n, seed, 2)
    if dtype == 0:
        m0 = m0.astype(np.float32).astype(np.float64)
    keys = ("Ms", "A", "D", "Ku", "eK", "Hbias", "alpha", "terms")
    op = Params(renorm=renorm, **{k: mat[k] for k in keys if k in mat})
    ref = omri.mri_run(g, op, m0, dt, dt_fast, nsteps, spec, P)
    ctx = magx.Context(n, d, dtype=dtype)
    t = torch.float32 if dtype == 0 else torch.float64
    m = torch.from_numpy(m0).to(device="cuda", dtype=t).contiguous()
    c0 = ctx.heff_count
    ctx.step_mri(m, magx.make_params(renorm=renorm, **mat), dt, nsteps, dt_fast)
    torch.cuda.synchronize()
    assert ctx.heff_count - c0 == 3 * nsteps
    return m.double().cpu().numpy(), ref, m0


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", [1, 0])
def test_one_mri_step_matches_oracle(name, dtype):
    got, ref, m0 = _run(name, dtype, 2, 1e-13, 1e-14, 1)
    assert _err(ref, m0) > 1e-4            # the step moves the state
    err = _err(got, ref)
    assert err <= (1e-11 if dtype == 1 else 1e-5), err


@pytest.mark.parametrize("renorm", [0, 1, 2])
def test_mri_steps_f64_renorm_modes(renorm):
    got, ref, _ = _run("tiny_all", 1, renorm, 8e-14, 1e-14, 4)
    assert _err(got, ref) <= 1e-11
    nrm = np.sqrt((got ** 2).sum(0))
    if renorm >= 1:
        assert np.abs(nrm - 1.0).max() < 1e-14


def test_mri_odd_stage_count_and_single_substep():
    # dt_fast >= dt: one substep per interval, 9 fast stages (odd: result ends in the workspace)
    got, ref, _ = _run("ragged_dmi", 1, 2, 5e-14, 1e-13, 3)
    assert _err(got, ref) <= 1e-11
    got, ref, _ = _run("ragged_dmi", 0, 2, 1e-13, 1e-14, 2)
    assert _err(got, ref) <= 2e-5


def test_mri_batched_equals_single():
    magx = _magx()
    n, d, mat = CASES["tiles"]
    p = magx.make_params(**mat)
    single = magx.Context(n, d, dtype=0)
    batch = magx.Context(n, d, dtype=0, nbatch=2)
    ms = [torch.from_numpy(random_unit_field(n, 820 + b, 2)).to(device="cuda", dtype=torch.float32)
          for b in range(2)]
    mB = torch.stack(ms).contiguous()
    batch.step_mri(mB, p, 1e-13, 2)
    for b in range(2):
        m = ms[b].clone()
        single.step_mri(m, p, 1e-13, 2)
        assert torch.equal(mB[b], m), b


def test_mri_bad_arguments():
    magx = _magx()
    n, d, mat = CASES["tiny_all"]
    ctx = magx.Context(n, d, dtype=1)
    m = torch.from_numpy(random_unit_field(n, 5, 2)).to(device="cuda").contiguous()
    m0 = m.clone()
    p = magx.make_params(**mat)
    for dt, dtf in ((1e-13, 0.0), (1e-13, -1.0), (math.nan, 1e-14), (1e-13, 1e-20)):
        with pytest.raises(magx.MagxError):
            ctx.step_mri(m, p, dt, 1, dtf)
    ctx.step_mri(m, p, 1e-13, 0)
    torch.cuda.synchronize()
    assert torch.equal(m, m0)
