"""Pins of the oracle's hand-written reverse mode against central finite
differences of the oracle's own forward map (FD with Richardson extrapolation;
the right-hand side is a cubic polynomial along any line, so the extrapolated
difference is exact up to rounding)."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import adjoint, llg, newell
from oracle.params import Grid, Params, TERM_DEMAG, TERM_EXCH, TERM_DMI, TERM_ANIS, TERM_ZEEMAN
from workloads import random_unit_field, random_vector_field, bernoulli_mask, tangent_direction

N = (5, 4, 3)
G = Grid(*N, 2e-9, 2e-9, 2e-9)


def _p(**kw):
    base = dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, eK=(0.0, 0.6, 0.8), alpha=0.1,
                Hbias=(2e4, -1e4, 3e4), terms=TERM_DEMAG | TERM_EXCH | TERM_DMI | TERM_ANIS | TERM_ZEEMAN)
    base.update(kw)
    return Params(**base)


def _fd(fun, eps):
    d1 = (fun(eps) - fun(-eps)) / (2 * eps)
    d2 = (fun(eps / 2) - fun(-eps / 2)) / eps
    return (4 * d2 - d1) / 3


@pytest.fixture(scope="module")
def spec():
    return newell.spectrum(G)


def test_vjp_rhs_matches_fd(spec):
    p = _p()
    y = random_unit_field(N, 31) * 1.1
    kappa = random_vector_field(N, 32)
    v = random_vector_field(N, 33)
    from oracle import field
    H = field.heff(G, p, y, spec)
    ybar, mu = adjoint.vjp_rhs(G, p, y, H, kappa, spec)
    fd = _fd(lambda e: float(np.sum(kappa * llg.rhs(G, p, y + e * v, spec))), 1e-3)
    assert abs(fd - float(np.sum(ybar * v))) < 1e-9 * abs(fd)
    # cotangent of the bias field
    for c in range(3):
        def f(e, c=c):
            h = list(p.Hbias)
            h[c] += e
            return float(np.sum(kappa * llg.rhs(G, replace(p, Hbias=tuple(h)), y, spec)))
        fdh = _fd(f, 100.0)
        assert abs(fdh - float(mu[c].sum())) < 1e-9 * max(abs(fdh), 1e-30) + 1e-18


def test_vjp_normalize_matches_fd():
    x = random_vector_field(N, 34)
    lam = random_vector_field(N, 35)
    v = random_vector_field(N, 36)
    got = float(np.sum(adjoint.vjp_normalize(x, lam) * v))
    fd = _fd(lambda e: float(np.sum(lam * llg.normalize(x + e * v)[0])), 1e-4)
    assert abs(got - fd) < 1e-7 * abs(fd)


@pytest.mark.parametrize("renorm", [0, 1, 2])
def test_step_vjp_matches_fd(spec, renorm):
    p = _p(renorm=renorm)
    m = random_unit_field(N, 37, smooth=1)
    lam = random_vector_field(N, 38)
    v = random_vector_field(N, 39)
    dt = 3e-14
    g, hb = adjoint.rk4_step_vjp(G, p, m, dt, lam, spec)
    fd = _fd(lambda e: float(np.sum(lam * llg.rk4_step(G, p, m + e * v, dt, spec))), 1e-4)
    assert abs(fd - float(np.sum(g * v))) < 1e-7 * abs(fd)
    for c in range(3):
        def f(e, c=c):
            h = list(p.Hbias)
            h[c] += e
            return float(np.sum(lam * llg.rk4_step(G, replace(p, Hbias=tuple(h)), m, dt, spec)))
        fdh = _fd(f, 10.0)
        assert abs(fdh - hb[c]) < 1e-6 * abs(fdh)


def test_rollout_gradient_matches_fd_and_is_checkpoint_invariant(spec):
    p = _p()
    m0 = random_unit_field(N, 40, smooth=3)
    mask = bernoulli_mask(N, 41)
    dt, nsteps = 5e-14, 6
    results = [adjoint.rollout_grad(G, p, m0, dt, nsteps, c, mask, spec) for c in (1, 2, 4, 6, 100)]
    loss, g, hb = results[0]
    for l2, g2, hb2 in results[1:]:
        assert l2 == loss
        assert np.array_equal(g2, g) and np.array_equal(hb2, hb)
    v = tangent_direction(m0, 42)

    def L(e):
        return adjoint.masked_mean_mz(mask, adjoint.rollout(G, p, m0 + e * v, dt, nsteps, spec))
    fd = _fd(L, 1e-5)
    assert abs(fd - float(np.sum(g * v))) < 1e-6 * abs(fd)

    def Lh(e):
        q = replace(p, Hbias=(p.Hbias[0], p.Hbias[1], p.Hbias[2] + e))
        return adjoint.masked_mean_mz(mask, adjoint.rollout(G, q, m0, dt, nsteps, spec))
    fdh = _fd(Lh, 10.0)
    assert abs(fdh - hb[2]) < 1e-6 * abs(fdh)
