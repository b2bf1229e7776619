"""Non-finite detection through the C ABI: calls made with check_finite = 1
clear a flag word in their workspace, every kernel that writes a field, a
state or a gradient sets it on a NaN or infinite output, and magx_status
reports it after waiting for the call's stream."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import random_unit_field  # noqa: E402

ENONFINITE = -6
MAT = dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, eK=(0.0, 0.0, 1.0), alpha=0.1, Hbias=(1e3, 0.0, 2e3), terms=31)


def _setup(n, dtype, terms=31):
    from paper_2602_12242_amd import magx
    ctx = magx.Context(n, (2e-9, 2e-9, 2e-9), dtype=dtype)
    mat = dict(MAT, terms=terms)
    p_on = magx.make_params(**mat, check_finite=1)
    p_off = magx.make_params(**mat, check_finite=0)
    m = torch.from_numpy(random_unit_field(n, 77, 1)).to("cuda", ctx.tdtype)
    return magx, ctx, p_on, p_off, m


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n,cell,terms", [((37, 11, 5), (36, 10, 4), 31), ((37, 11, 5), (17, 3, 2), 2 | 4 | 8),
                                          ((64, 16, 2), (5, 0, 1), 2), ((128, 32, 1), (0, 0, 0), 31)])
def test_nan_in_state_is_reported(dtype, n, cell, terms):
    # the poisoned cell: the last one of an odd row (a single-cell pair), an
    # interior one, an odd x of an even row; without demag the NaN stays in
    # the stencil's reach, with it the FFT spreads it everywhere
    magx, ctx, p_on, p_off, m = _setup(n, dtype, terms)
    dt = 1e-13
    print(f"status case n={n} cell={cell} terms={terms} dtype={dtype}", flush=True)
    y = m.clone()
    ctx.step(y, p_on, dt, 2)
    assert ctx.status() == 0
    ctx.heff(m, p_on)
    assert ctx.status() == 0
    bad = m.clone()
    x, yy, z = cell
    bad[1, z, yy, x] = float("nan")
    y = bad.clone()
    ctx.step(y, p_on, dt, 1)
    assert ctx.status() == ENONFINITE
    # a clean checked call clears the flag; an unchecked call leaves it alone
    y = m.clone()
    ctx.step(y, p_on, dt, 1)
    assert ctx.status() == 0
    y = bad.clone()
    ctx.step(y, p_off, dt, 1)
    assert ctx.status() == 0
    ctx.heff(bad, p_on)
    assert ctx.status() == ENONFINITE
    ctx.step_euler(m.clone(), p_on, dt, 1)
    assert ctx.status() == 0
    ctx.step_euler(bad.clone(), p_on, dt, 1)
    assert ctx.status() == ENONFINITE
    ctx.step_mri(bad.clone(), p_on, dt, 1)
    assert ctx.status() == ENONFINITE
    e = ctx.energy(bad, p_on)
    assert ctx.status() == ENONFINITE
    assert not bool(torch.isfinite(e[5]))


@pytest.mark.parametrize("dtype", [0, 1])
def test_infinite_gradient_is_reported(dtype):
    magx, ctx, p_on, p_off, m = _setup((37, 11, 5), dtype)
    dt = 1e-13
    tape = ctx.tape(2)
    y = m.clone()
    ctx.step(y, p_on, dt, 2, tape=tape)
    assert ctx.status() == 0
    gm = torch.zeros_like(m)
    gm[2] = 1.0 / gm[2].numel()
    gh = torch.zeros(3, dtype=ctx.tdtype, device="cuda")
    ctx.step_backward(tape, 2, p_on, dt, gm.clone(), gh)
    assert ctx.status() == 0
    gbad = gm.clone()
    gbad[0, 2, 5, 9] = float("inf")
    ctx.step_backward(tape, 2, p_on, dt, gbad, gh)
    assert ctx.status() == ENONFINITE
    ctx.heff_backward(gbad, p_on)
    assert ctx.status() == ENONFINITE
    ctx.heff_backward(gm, p_on)
    assert ctx.status() == 0


def test_rollout_counts_as_one_checked_call():
    # a NaN met in the first segment of a checkpointed rollout is still
    # reported after the later segments ran
    magx, ctx, p_on, p_off, m = _setup((37, 11, 5), 0)
    bad = m.clone()
    bad[0, 0, 0, 0] = float("nan")
    store = ctx.checkpoint_store(6, 2)
    ctx.rollout_forward(bad, p_on, 1e-13, 6, 2, store)
    assert ctx.status() == ENONFINITE
    y = m.clone()
    ctx.rollout_forward(y, p_on, 1e-13, 6, 2, store)
    assert ctx.status() == 0
    gm = torch.zeros_like(m)
    gm[2] = 1.0
    ctx.rollout_backward(store, p_on, 1e-13, 6, 2, gm)
    assert ctx.status() == 0
    assert math.isfinite(float(gm.abs().sum()))


def test_memory_probe_patterns():
    # the diagnostic memory patterns run over the workspace and report the
    # bytes they move: the copy moves the X2 region once, the tilings read and
    # write every stored column of every row
    from paper_2602_12242_amd import magx
    n = (37, 11, 5)
    ctx = magx.Context(n, (2e-9, 2e-9, 2e-9), dtype=0)
    Px, Py, Pz = 128, 32, 16
    Hx = Px // 2 + 1
    Sx = (Hx + 15) // 16 * 16
    assert ctx.memory_probe(0) == 3 * n[2] * Py * Sx * 8
    assert ctx.memory_probe(1) == 2 * 3 * n[2] * Py * Hx * 8
    assert ctx.memory_probe(2) == 2 * 3 * n[2] * Py * Hx * 8
    torch.cuda.synchronize()
    with pytest.raises(magx.MagxError):
        magx.Context(n, (2e-9, 2e-9, 2e-9), dtype=1).memory_probe(0)
