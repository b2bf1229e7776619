"""Batched systems sharing one tensor spectrum, through the C ABI.

A context of B members must give each member exactly (bit for bit) what a
one-system context gives it: the batch only changes which blocks of one launch
work on which member, never the arithmetic or its order.  One member is also
compared with the FP64 oracle directly.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import field as ofield  # noqa: E402
from oracle import newell as onewell  # noqa: E402
from oracle.params import Grid, Params  # noqa: E402
from workloads import random_unit_field, random_vector_field  # noqa: E402

ALL = 31
CASES = {
    "tiny_all": ((7, 5, 3), (2e-9, 2.5e-9, 1.5e-9),
                 dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, eK=(0.0, 0.6, 0.8), alpha=0.1,
                      Hbias=(2e4, -1e4, 3e4), terms=ALL)),
    "ragged_dmi": ((37, 11, 5), (2e-9, 2e-9, 2e-9),
                   dict(Ms=1.1e6, A=1.6e-11, D=3e-3, Ku=1e6, eK=(0, 0, 1), alpha=0.3, Hbias=(0, 0, 1e4),
                        terms=ALL)),
    "tiles": ((96, 70, 9), (2e-9, 2e-9, 3e-9),
              dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, alpha=0.1, Hbias=(1e3, 2e3, -5e3), terms=ALL)),
    # Pz = 64: the register-resident z pass (single precision) walks units of
    # every member
    "thick": ((40, 9, 20), (2e-9, 2e-9, 1e-9),
              dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, eK=(0.6, 0.0, 0.8), alpha=0.1, Hbias=(1e3, -2e3, 5e3),
                   terms=ALL)),
    # square power-of-two plane: compile-time pencil and y geometry
    "sq128": ((128, 128, 2), (2e-9, 2e-9, 2e-9),
              dict(Ms=8e5, A=1.3e-11, D=1e-3, alpha=0.1, Hbias=(2e3, 0, 1e3), terms=ALL)),
    # a film (nz = 1): the fused y and z passes take column tiles of every member
    "film": ((100, 24, 1), (3e-9, 3e-9, 3e-9),
             dict(Ms=8e5, A=1.3e-11, D=1e-3, alpha=0.02, Hbias=(2e4, 0, 0), terms=ALL)),
    # Pz = 128: the single-precision z pass with 16 threads per column and the
    # double-precision one with 32 (tensor blocks copied to LDS per tile)
    "slab40": ((20, 6, 40), (2e-9, 2e-9, 1e-9),
               dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, eK=(0.0, 0.6, 0.8), alpha=0.1, Hbias=(1e3, -2e3, 5e3),
                    terms=ALL)),
}
B = 3


def _magx():
    from paper_2602_12242_amd import magx
    return magx


def _states(n, dtype, seed0):
    t = torch.float32 if dtype == 0 else torch.float64
    ms = [torch.from_numpy(random_unit_field(n, seed0 + b, 2)).to(device="cuda", dtype=t) for b in range(B)]
    return ms, torch.stack(ms).contiguous()


def _biases(mat):
    base = np.asarray(mat["Hbias"], dtype=np.float64)
    return [base * (1.0 + 0.5 * b) + np.array([3e3 * b, -2e3 * b, 1e3]) for b in range(B)]


def _params_with_bias(mat, h):
    magx = _magx()
    q = dict(mat)
    q["Hbias"] = tuple(float(v) for v in h)
    return magx.make_params(**q)


def _setup(name, dtype):
    magx = _magx()
    n, d, mat = CASES[name]
    single = magx.Context(n, d, dtype=dtype)
    batch = magx.Context(n, d, dtype=dtype, nbatch=B)
    assert batch.shape == (B, 3, n[2], n[1], n[0])
    assert batch.lib.magx_ctx_batch(batch.h) == B
    hs = _biases(mat)
    hb = torch.tensor(np.stack(hs), dtype=batch.tdtype, device="cuda").contiguous()
    # the device copy of each bias must be what the context type makes of the double
    pb = [_params_with_bias(mat, hb[b].double().cpu().numpy()) for b in range(B)]
    batch.set_member_bias(hb)
    return n, d, mat, single, batch, pb


def _same(a, b):
    return torch.equal(a, b)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", [0, 1])
def test_batched_heff_energy_rhs_equal_single(name, dtype):
    n, d, mat, single, batch, pb = _setup(name, dtype)
    p = _magx().make_params(**mat)
    ms, mB = _states(n, dtype, 700)
    HB = batch.heff(mB, p)
    EB = batch.energy(mB, p)
    kB = batch.llg_rhs(mB, HB, p)
    for b in range(B):
        H = single.heff(ms[b], pb[b])
        assert _same(HB[b], H), b
        assert _same(EB[b], single.energy(ms[b], pb[b])), b
        assert _same(kB[b], single.llg_rhs(ms[b], H, pb[b])), b


@pytest.mark.parametrize("name", ["tiny_all", "tiles", "film", "slab40"])
def test_batched_member_matches_oracle(name):
    n, d, mat, single, batch, pb = _setup(name, 1)
    p = _magx().make_params(**mat)
    ms, mB = _states(n, 1, 710)
    HB = batch.heff(mB, p).cpu().numpy()
    g = Grid(*n, *d)
    P = tuple(max(2, 1 << (2 * v - 1).bit_length()) for v in (n[2], n[1], n[0]))
    spec = onewell.spectrum(g, P)
    keys = ("Ms", "A", "D", "Ku", "eK", "alpha", "terms")
    for b in range(B):
        h = batch.member_bias[b].cpu().numpy()
        op = Params(Hbias=tuple(h), **{k: mat[k] for k in keys if k in mat})
        ref = ofield.heff(g, op, ms[b].cpu().numpy(), spec, P)
        err = np.sqrt(((HB[b] - ref) ** 2).sum(0)).max() / np.sqrt((ref ** 2).sum(0)).max()
        assert err <= 1e-11, (b, err)


@pytest.mark.parametrize("name", ["tiny_all", "ragged_dmi", "tiles", "thick", "sq128", "film", "slab40"])
@pytest.mark.parametrize("dtype", [0, 1])
def test_batched_steps_and_reverse_equal_single(name, dtype):
    n, d, mat, single, batch, pb = _setup(name, dtype)
    p = _magx().make_params(**mat)
    dt, nsteps = 5e-14, 3
    ms, mB = _states(n, dtype, 720)
    tapeB = batch.tape(nsteps)
    batch.step(mB, p, dt, nsteps, tapeB)
    gB = torch.from_numpy(np.stack([random_vector_field(n, 730 + b) for b in range(B)])).to(
        device="cuda", dtype=batch.tdtype).contiguous()
    g0 = gB.clone()
    ghB = torch.zeros((B, 3), dtype=batch.tdtype, device="cuda")
    batch.step_backward(tapeB, nsteps, p, dt, gB, ghB)
    for b in range(B):
        m = ms[b].clone()
        tape = single.tape(nsteps)
        single.step(m, pb[b], dt, nsteps, tape)
        assert _same(mB[b], m), b
        g = g0[b].clone().contiguous()
        gh = torch.zeros(3, dtype=single.tdtype, device="cuda")
        single.step_backward(tape, nsteps, pb[b], dt, g, gh)
        assert _same(gB[b], g), b
        assert _same(ghB[b], gh), b


def test_batched_checkpointed_rollout_equals_single():
    n, d, mat, single, batch, pb = _setup("tiles", 0)
    p = _magx().make_params(**mat)
    dt, nsteps, ckpt = 5e-14, 5, 2
    ms, mB = _states(n, 0, 740)
    store = batch.checkpoint_store(nsteps, ckpt)
    batch.rollout_forward(mB, p, dt, nsteps, ckpt, store)
    gB = torch.from_numpy(np.stack([random_vector_field(n, 750 + b) for b in range(B)])).to(
        device="cuda", dtype=torch.float32).contiguous()
    g0 = gB.clone()
    gB, ghB = batch.rollout_backward(store, p, dt, nsteps, ckpt, gB)
    for b in range(B):
        m = ms[b].clone()
        st = single.checkpoint_store(nsteps, ckpt)
        single.rollout_forward(m, pb[b], dt, nsteps, ckpt, st)
        assert _same(mB[b], m), b
        g, gh = single.rollout_backward(st, pb[b], dt, nsteps, ckpt, g0[b].clone().contiguous())
        assert _same(gB[b], g), b
        assert _same(ghB[b], gh), b


def test_member_bias_reset_and_validation():
    magx = _magx()
    n, d, mat, single, batch, pb = _setup("tiny_all", 1)
    p = magx.make_params(**mat)
    ms, mB = _states(n, 1, 760)
    batch.set_member_bias(None)
    HB = batch.heff(mB, p)
    for b in range(B):
        assert _same(HB[b], single.heff(ms[b], p)), b
    with pytest.raises(ValueError):
        batch.set_member_bias(torch.zeros((B + 1, 3), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        batch.heff(ms[0], p)
    assert math.isfinite(float(HB.abs().max()))
