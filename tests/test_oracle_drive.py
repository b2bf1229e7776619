"""Pins of forward Euler and of the time-dependent bias field (oracle), from
the closed-form motion of a single cell in a field along a fixed axis.

Eq. (1) for one cell with H(t) = h(t) e_z, in spherical angles of m:
  theta' = a alpha h sin(theta),  phi' = -a h,   a = mu0 gamma / (1 + alpha^2)
so with I(t) = integral of h from 0 to t:
  tan(theta/2) = tan(theta0/2) exp(a alpha I(t)),  phi = phi0 - a I(t).
This holds for any h(t), so a linear ramp checks that every stage of a
method sees the bias at its own time: evaluated at the step start instead,
RK4 drops to first order.
"""
import math

import numpy as np
import pytest

from oracle import llg as ollg
from oracle import mri as omri
from oracle.params import Grid, Params

GRID = Grid(1, 1, 1, 2e-9, 2e-9, 2e-9)
ALPHA = 0.3
H0, H1 = 2.0e5, 4.0e16          # A/m and A/(m s): the ramp doubles h in 5 ps
TH0, PH0 = 2.2, 0.4


def _p(renorm=0):
    return Params(Ms=8e5, alpha=ALPHA, terms=16, Hbias=(0.0, 0.0, H0), renorm=renorm)


def _m0():
    return np.array([math.sin(TH0) * math.cos(PH0), math.sin(TH0) * math.sin(PH0),
                     math.cos(TH0)]).reshape(3, 1, 1, 1)


def _exact(I, p):
    a = ollg.prefactor(p)
    th = 2.0 * math.atan(math.tan(TH0 / 2.0) * math.exp(a * ALPHA * I))
    ph = PH0 - a * I
    return np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])


def _ramp():
    # knots far enough apart that the interpolation is the exact line over [0, T]
    return ollg.bias_schedule([0.0, 1e-10], [(0, 0, H0), (0, 0, H0 + H1 * 1e-10)])


def _orders(errs):
    return [math.log2(e0 / e1) for e0, e1 in zip(errs, errs[1:])]


T = 5e-12


def test_schedule_interpolates_and_clamps():
    at = ollg.bias_schedule([1.0, 3.0, 4.0], [(0, 0, 0), (2, 4, 6), (2, 0, 6)])
    assert np.allclose(at(0.0), (0, 0, 0)) and np.allclose(at(1.0), (0, 0, 0))
    assert np.allclose(at(2.0), (1, 2, 3))
    assert np.allclose(at(3.5), (2, 2, 6))
    assert np.allclose(at(9.0), (2, 0, 6))


def test_closed_form_itself():
    # the formula satisfies the ODE: compare its finite-difference derivative
    # with Eq. (1) at a point of the ramp
    p = _p()
    t, h = 2e-12, 1e-16
    I = lambda s: H0 * s + 0.5 * H1 * s * s  # noqa: E731
    dm = (_exact(I(t + h), p) - _exact(I(t - h), p)) / (2 * h)
    m = _exact(I(t), p)
    H = np.array([0.0, 0.0, H0 + H1 * t])
    rhs = ollg.rhs_from_field(p, m.reshape(3, 1, 1, 1), H.reshape(3, 1, 1, 1)).ravel()
    assert np.abs(dm - rhs).max() < 1e-6 * np.abs(rhs).max()


@pytest.mark.parametrize("renorm", [0, 1])
def test_euler_is_first_order(renorm):
    p = _p(renorm)
    ex = _exact(H0 * T, p)
    errs = []
    for n in (200, 400, 800):
        m = _m0()
        for _ in range(n):
            m = ollg.euler_step(GRID, p, m, T / n)
        errs.append(np.abs(m.ravel() - ex).max())
    o = _orders(errs)
    assert all(0.9 < v < 1.1 for v in o), o


def test_rk4_with_a_ramped_bias_is_fourth_order():
    p = _p()
    at = _ramp()
    ex = _exact(H0 * T + 0.5 * H1 * T * T, p)
    errs = []
    for n in (10, 20, 40):
        m, dt = _m0(), T / n
        for k in range(n):
            m = ollg.rk4_step(GRID, p, m, dt, t0=k * dt, bias_at=at)
        errs.append(np.abs(m.ravel() - ex).max())
    o = _orders(errs)
    assert min(o) > 3.7, (errs, o)


def test_bias_frozen_at_the_step_start_is_only_first_order():
    # the plausible mistake the stage-time evaluation guards against
    p = _p()
    at = _ramp()
    ex = _exact(H0 * T + 0.5 * H1 * T * T, p)
    errs = []
    for n in (10, 20, 40):
        m, dt = _m0(), T / n
        for k in range(n):
            m = ollg.rk4_step(GRID, ollg.with_bias(p, at(k * dt)), m, dt)
        errs.append(np.abs(m.ravel() - ex).max())
    assert max(_orders(errs)) < 1.5


def test_euler_with_a_ramped_bias_is_first_order():
    p = _p(1)
    at = _ramp()
    ex = _exact(H0 * T + 0.5 * H1 * T * T, p)
    errs = []
    for n in (200, 400, 800):
        m, dt = _m0(), T / n
        for k in range(n):
            m = ollg.euler_step(GRID, p, m, dt, t0=k * dt, bias_at=at)
        errs.append(np.abs(m.ravel() - ex).max())
    o = _orders(errs)
    assert all(0.9 < v < 1.1 for v in o), o


def test_multirate_with_a_ramped_bias_is_third_order():
    # one cell has no exchange: the fast partition is zero and the multirate
    # step is the Knoth-Wolke method on the slow (bias) torque
    p = _p()
    at = _ramp()
    ex = _exact(H0 * T + 0.5 * H1 * T * T, p)
    errs = []
    for n in (10, 20, 40):
        dt = T / n
        m = omri.mri_run(GRID, p, _m0(), dt, dt / 10, n, bias_at=at)
        errs.append(np.abs(m.ravel() - ex).max())
    o = _orders(errs)
    assert min(o) > 2.8, (errs, o)
