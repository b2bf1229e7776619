"""Small grids step through replayed HIP graphs (magx_step without a tape):
the replays must give the directly launched results bit for bit (a taped
step launches directly and computes the same values), on repeated calls
with other work and synchronisations in between, for chunked step counts,
batches, both precisions and with the non-finite check."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import WORKLOADS, initial_state, random_unit_field  # noqa: E402

MAT = dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, eK=(0.0, 0.6, 0.8), alpha=0.1, Hbias=(2e4, -1e4, 3e4), terms=31)


def _direct(ctx, m0, p, dt, n):
    # a taped step is never replayed from a graph
    a = m0.clone()
    ctx.step(a, p, dt, n, tape=ctx.tape(n))
    return a


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("case", ["film", "ragged"])
def test_graph_replays_equal_direct_launches(dtype, case):
    from paper_2602_12242_amd import magx
    if case == "film":
        w = WORKLOADS["film"]
        n, d, mat, dt = w.n, w.d, w.material(), w.dt
        m0h = initial_state(w)
    else:
        n, d, mat, dt = (37, 11, 5), (2e-9, 2.5e-9, 1.5e-9), MAT, 1e-13
        m0h = random_unit_field(n, 31, 2).astype("float32")
    print(f"graph case {case} dtype={dtype}", flush=True)
    ctx = magx.Context(n, d, dtype=dtype)
    p = magx.make_params(**mat)
    m0 = torch.from_numpy(m0h).to("cuda", ctx.tdtype)
    for nsteps in (1, 5, 16, 21, 40):
        ref = _direct(ctx, m0, p, dt, nsteps)
        for rep in range(3):
            before = ctx.heff_count
            b = m0.clone()
            ctx.step(b, p, dt, nsteps)              # replayed (captured on the first call)
            torch.cuda.synchronize()
            assert ctx.heff_count - before == 4 * nsteps
            assert torch.equal(b, ref), (nsteps, rep)
            # other work on the stream between replays
            ctx.heff(b, p)
            _ = _direct(ctx, b, p, dt, 1)
    # the same graph on another buffer and after a parameter change
    c = m0.clone()
    ctx.step(c, p, dt, 5)
    assert torch.equal(c, _direct(ctx, m0, p, dt, 5))
    q = magx.make_params(**dict(mat, alpha=0.3))
    e = m0.clone()
    ctx.step(e, q, dt, 5)
    assert torch.equal(e, _direct(ctx, m0, q, dt, 5))
    assert not torch.equal(e, c)


def test_graph_batched_and_checked():
    from paper_2602_12242_amd import magx
    w = WORKLOADS["film"]
    B = 4
    ctx = magx.Context(w.n, w.d, dtype=0, nbatch=B)
    import numpy as np
    m0 = torch.from_numpy(np.stack([random_unit_field(w.n, 500 + b, 3) for b in range(B)])).to(
        "cuda", torch.float32).contiguous()
    p = magx.make_params(**w.material(), check_finite=1)
    ref = _direct(ctx, m0, p, w.dt, 7)
    for _ in range(3):
        b = m0.clone()
        ctx.step(b, p, w.dt, 7)
        assert ctx.status() == 0
        assert torch.equal(b, ref)
    bad = m0.clone()
    bad[2, 1, 0, 0, 5] = float("nan")
    ctx.step(bad, p, w.dt, 7)
    assert ctx.status() == -6
    b = m0.clone()
    ctx.step(b, p, w.dt, 7)
    assert ctx.status() == 0
