"""GPU parity at the workloads' full sizes, in the launch configurations the
benchmark times (Section II-B convolution, Eq. (2) field, RK4 of Section
III-C, and the reverse mode), against the FP64 oracle:

* 256 x 256 x 8 (adjoint workload) and 256 x 256 x 16 (DMI workload): H_eff
  and one RK4 step element by element over every cell, and at 256 x 256 x 8
  the vector-Jacobian product of one step;
* 512 x 512 x 32 (demag workload): H_eff and one RK4 step at 4096 seeded cells
  plus the box's corners and face centres, stored by
  tests/golden/make_workload_golden.py (oracle only);
* the adjoint workload as configured: 100 steps, checkpoint every 10, loss =
  masked mean of m_z; the gradient's projections on 64 seeded tangent
  directions and dL/dH_bias against central differences of the FP64 forward
  map and against the oracle's reverse sweep (stored by the same script);
* 1024 x 1024 x 64 (large workload): 50 steps forward + checkpointed adjoint
  in FP32 against the FP64 GPU path (the oracle does not fit this grid).

Errors: fields normwise, max_i |a_i - b_i| / max_i |b_i|; states absolute
(|m| = 1); gradients as || (g . v_k - ref_k)_k || / || (ref_k)_k || over the
directions.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import adjoint as oadj  # noqa: E402
from oracle import field as ofield  # noqa: E402
from oracle import llg as ollg  # noqa: E402
from oracle import newell as onewell  # noqa: E402
from oracle.params import Grid, Params  # noqa: E402
from workloads import WORKLOADS, bernoulli_mask, initial_state, random_vector_field, tangent_direction  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_ORACLE = {}


def _oparams(mat):
    return Params(**{k: mat[k] for k in ("Ms", "A", "D", "Ku", "eK", "Hbias", "alpha", "terms", "renorm")})


def _gparams(mat, **over):
    from paper_2602_12242_amd import magx
    d = dict(mat)
    d.update(over)
    return magx.make_params(**d)


def _ctx(w, dtype):
    from paper_2602_12242_amd import magx
    return magx.Context(w.n, w.d, dtype=dtype)


def _err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(((a - b) ** 2).sum(0)).max() / np.sqrt((b ** 2).sum(0)).max())


def _free(*objs):
    for o in objs:
        del o
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _oracle(name):
    """Oracle spectrum, H_eff and one RK4 step of a workload's initial state (cached)."""
    if name not in _ORACLE:
        w = WORKLOADS[name]
        g = Grid(*w.n, *w.d)
        spec = onewell.spectrum(g)
        op = _oparams(w.material())
        m = initial_state(w).astype(np.float64)
        H = ofield.heff(g, op, m, spec)
        m1 = ollg.rk4_step(g, op, m, w.dt, spec)
        _ORACLE[name] = dict(g=g, spec=spec, op=op, H=H, m1=m1)
    return _ORACLE[name]


@pytest.mark.parametrize("name", ["adjoint", "dmi"])
@pytest.mark.parametrize("dtype", [1, 0])
def test_workload_heff_and_step_match_oracle_every_cell(name, dtype):
    w = WORKLOADS[name]
    print(f"workload parity: {name} {w.n} dtype={dtype}", flush=True)
    o = _oracle(name)
    m = initial_state(w)
    ctx = _ctx(w, dtype)
    p = _gparams(w.material())
    mg = torch.from_numpy(m).to("cuda", ctx.tdtype)
    H = ctx.heff(mg, p).cpu().numpy()
    errH = _err(H, o["H"])
    ctx.step(mg, p, w.dt, 1)
    errm = float(np.abs(mg.cpu().numpy() - o["m1"]).max())
    print(f"  err_H {errH:.3e}  err_m(1 step) {errm:.3e}", flush=True)
    assert errH <= (1e-11 if dtype == 1 else 1e-5)
    assert errm <= (1e-11 if dtype == 1 else 1e-5)
    _free(ctx, mg)


@pytest.mark.parametrize("dtype", [1, 0])
def test_adjoint_workload_step_vjp_matches_oracle_every_cell(dtype):
    w = WORKLOADS["adjoint"]
    print(f"workload step VJP: adjoint {w.n} dtype={dtype}", flush=True)
    o = _oracle("adjoint")
    m = initial_state(w)
    lam = random_vector_field(w.n, 109)
    if "vjp" not in o:
        o["vjp"] = oadj.rk4_step_vjp(o["g"], o["op"], m.astype(np.float64), w.dt, lam, o["spec"])
    ref, refh = o["vjp"]
    ctx = _ctx(w, dtype)
    p = _gparams(w.material())
    mg = torch.from_numpy(m).to("cuda", ctx.tdtype)
    tape = ctx.tape(1)
    ctx.step(mg, p, w.dt, 1, tape=tape)
    gm = torch.from_numpy(lam).to("cuda", ctx.tdtype)
    gh = torch.zeros(3, dtype=ctx.tdtype, device="cuda")
    ctx.step_backward(tape, 1, p, w.dt, gm, gh)
    err = _err(gm.cpu().numpy(), ref)
    errh = float(np.abs(gh.cpu().numpy() - refh).max() / np.abs(refh).max())
    print(f"  err_grad {err:.3e}  err_dHbias {errh:.3e}", flush=True)
    tol = 1e-10 if dtype == 1 else 1e-4
    assert err <= tol and errh <= tol
    _free(ctx, tape, gm)


@pytest.mark.parametrize("dtype", [1, 0])
def test_demag_workload_matches_stored_oracle_cells(dtype):
    w = WORKLOADS["demag"]
    gold = np.load(os.path.join(GOLDEN, "demag512_sampled.npz"))
    assert int(gold["seed"]) == w.seed and float(gold["dt"]) == w.dt
    x, y, z = gold["cells"].T
    print(f"workload parity: demag {w.n} dtype={dtype}, {len(x)} stored cells", flush=True)
    ctx = _ctx(w, dtype)
    p = _gparams(w.material())
    mg = torch.from_numpy(initial_state(w)).to("cuda", ctx.tdtype)
    H = ctx.heff(mg, p)
    Hs = H[:, z, y, x].T.double().cpu().numpy()
    errH = float(np.sqrt(((Hs - gold["H"]) ** 2).sum(1)).max() / float(gold["hmax"]))
    ctx.step(mg, p, w.dt, 1)
    ms = mg[:, z, y, x].T.double().cpu().numpy()
    errm = float(np.abs(ms - gold["m1"]).max())
    print(f"  err_H {errH:.3e}  err_m(1 step) {errm:.3e}", flush=True)
    assert errH <= (1e-11 if dtype == 1 else 1e-5)
    assert errm <= (1e-11 if dtype == 1 else 1e-5)
    _free(ctx, H, mg)


def _loss_and_grad(ctx, w, p, m0, mask, nsteps, ckpt, hbias=None):
    from paper_2602_12242_amd import magx
    m = m0.clone().requires_grad_(True)
    hb = w.material()["Hbias"] if hbias is None else hbias
    h = torch.tensor(hb, dtype=m.dtype, device="cuda", requires_grad=True)
    mT = magx.Rollout.apply(m, h, ctx, p, w.dt, nsteps, ckpt)
    L = (mask * mT[2]).sum() / mask.sum()
    L.backward()
    return float(L.detach()), m.grad.detach(), h.grad.detach().double().cpu().numpy()


def _proj_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_adjoint_workload_gradient_fd_oracle_and_precision():
    # the adjoint workload as configured: 100 RK4 steps of 5e-14 s, checkpoint
    # every 10 steps; FD of the float64 forward map along the 64 seeded tangent
    # directions (eps 1e-5) and along each axis of H_bias (eps 10 A/m)
    w = WORKLOADS["adjoint"]
    gold = np.load(os.path.join(GOLDEN, "adjoint256_grad.npz"))
    nsteps, ckpt = w.steps, w.ckpt
    assert int(gold["steps"]) == nsteps and int(gold["ckpt"]) == ckpt
    m0 = torch.from_numpy(initial_state(w)).cuda()
    mask = torch.from_numpy(bernoulli_mask(w.n, w.extra["mask_seed"])).cuda()
    m0d = m0.double().cpu().numpy()
    dirs = [tangent_direction(m0d, int(s)) for s in gold["seeds"]]
    print(f"adjoint workload: {nsteps} steps, ckpt {ckpt}, {len(dirs)} FD directions", flush=True)
    c64 = _ctx(w, 1)
    p = _gparams(w.material())
    L64, g64, h64 = _loss_and_grad(c64, w, p, m0.double(), mask.double(), nsteps, ckpt)

    def loss64(m, q):
        m = m.contiguous()
        c64.step(m, q, w.dt, nsteps)
        return float((mask.double() * m[2]).sum() / mask.sum())

    # central differences at eps and 2 eps: the first is the stated check, the
    # fourth-order combination (4 D(eps) - D(2 eps)) / 3 removes the O(eps^2)
    # truncation error that dominates the first in FP64
    eps = 1e-5
    fd, fd4 = [], []
    for v in dirs:
        vg = torch.from_numpy(v).cuda()
        d1 = (loss64(m0.double() + eps * vg, p) - loss64(m0.double() - eps * vg, p)) / (2 * eps)
        d2 = (loss64(m0.double() + 2 * eps * vg, p) - loss64(m0.double() - 2 * eps * vg, p)) / (4 * eps)
        fd.append(d1)
        fd4.append((4 * d1 - d2) / 3)
    fd = np.array(fd)
    fd4 = np.array(fd4)
    hb0 = np.array(w.material()["Hbias"], dtype=np.float64)
    fdh = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = 10.0
        fdh.append((loss64(m0.double(), _gparams(w.material(), Hbias=tuple(hb0 + e)))
                    - loss64(m0.double(), _gparams(w.material(), Hbias=tuple(hb0 - e)))) / 20.0)
    fdh = np.array(fdh)
    an64 = np.array([float((g64 * torch.from_numpy(v).cuda()).sum()) for v in dirs])
    _free(c64, g64)
    c32 = _ctx(w, 0)
    L32, g32, h32 = _loss_and_grad(c32, w, p, m0, mask.float(), nsteps, ckpt)
    an32 = np.array([float((g32.double() * torch.from_numpy(v).cuda()).sum()) for v in dirs])
    res = dict(fd64=_proj_err(an64, fd), fd4_64=_proj_err(an64, fd4), oracle64=_proj_err(an64, gold["proj"]),
               fd32=_proj_err(an32, fd), oracle32=_proj_err(an32, gold["proj"]),
               h64_fd=_proj_err(h64, fdh), h64_oracle=_proj_err(h64, gold["gHbias"]),
               h32_fd=_proj_err(h32, fdh), h32_oracle=_proj_err(h32, gold["gHbias"]),
               loss64=abs(L64 - float(gold["loss"])), loss32=abs(L32 - float(gold["loss"])))
    print("  " + "  ".join(f"{k} {v:.2e}" for k, v in res.items()), flush=True)
    # FP64 GPU reverse mode = oracle reverse sweep (same algorithm, other rounding)
    assert res["oracle64"] <= 1e-9 and res["h64_oracle"] <= 1e-9 and res["loss64"] <= 1e-12
    # the gradient is the derivative of the forward map: central FD within the
    # stated 1e-4 (its O(eps^2) truncation is ~6e-6 here), fourth-order FD closer
    assert res["fd64"] <= 1e-4 and res["fd4_64"] <= 1e-7 and res["h64_fd"] <= 1e-6
    # single precision within 1e-4 of both
    assert res["fd32"] <= 1e-4 and res["oracle32"] <= 1e-4
    assert res["h32_fd"] <= 1e-4 and res["h32_oracle"] <= 1e-4
    assert res["loss32"] <= 1e-6
    _free(c32, g32)


def test_large_workload_forward_and_adjoint_f32_vs_f64():
    # 1024 x 1024 x 64, 50 RK4 steps forward and the checkpointed adjoint of
    # the masked-mean-m_z loss; FP64 with checkpoints every 5 steps (its tape
    # of 5 steps is 75 GB), FP32 every 10
    w = WORKLOADS["large"]
    nsteps = w.steps
    m0 = torch.from_numpy(initial_state(w)).cuda()
    mask = torch.from_numpy(bernoulli_mask(w.n, w.extra["mask_seed"])).cuda()
    seeds = (3100, 3101, 3102, 3103)
    print(f"large workload: {w.n}, {nsteps} steps fwd + adjoint, FP64 first", flush=True)
    c64 = _ctx(w, 1)
    p = _gparams(w.material())
    L64, g64, h64 = _loss_and_grad(c64, w, p, m0.double(), mask.double(), nsteps, 5)
    m64 = m0.double().clone()
    c64.step(m64, p, w.dt, nsteps)
    m64 = m64.cpu()
    dirs = [torch.from_numpy(tangent_direction(m0.double().cpu().numpy(), s)) for s in seeds]
    an64 = np.array([float((g64.cpu() * v).sum()) for v in dirs])
    g64c = g64.cpu()
    _free(c64, g64)
    c32 = _ctx(w, 0)
    L32, g32, h32 = _loss_and_grad(c32, w, p, m0, mask.float(), nsteps, w.ckpt)
    m32 = m0.clone()
    c32.step(m32, p, w.dt, nsteps)
    errm = float((m32.cpu().double() - m64).abs().max())
    an32 = np.array([float((g32.cpu().double() * v).sum()) for v in dirs])
    errg = _err(g32.cpu().double().numpy(), g64c.numpy())
    res = dict(err_m=errm, loss=abs(L32 - L64), proj=_proj_err(an32, an64), grad_cells=errg,
               hbias=_proj_err(h32, h64))
    print("  " + "  ".join(f"{k} {v:.2e}" for k, v in res.items()), flush=True)
    assert res["err_m"] <= 1e-4 and res["loss"] <= 1e-6
    assert res["proj"] <= 1e-4 and res["hbias"] <= 1e-4
    assert res["grad_cells"] <= 1e-4
    _free(c32, g32)
