"""Pins of the multirate oracle (Section III-C, explicit-explicit MRI with the
Knoth-Wolke method on both time scales) against facts that do not come from
the oracle itself: the published low-storage form of the same method,
closed-form solutions, convergence orders and the reductions of the
multirate step to single-rate stepping."""
from fractions import Fraction as Fr
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import llg as ollg
from oracle import mri as omri
from oracle import newell as onewell
from oracle.params import Grid, Params
from workloads import random_unit_field


def test_table_equals_williamson_low_storage_form():
    # Williamson's three-stage 2N-storage scheme, q <- A_k q + h f, y <- y + B_k q,
    # with A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15), is the same method.
    # Expand it symbolically: coefficient vectors over the stage derivatives.
    Aw = (Fr(0), Fr(-5, 9), Fr(-153, 128))
    Bw = (Fr(1, 3), Fr(15, 16), Fr(8, 15))
    q = [Fr(0)] * 3
    y = [Fr(0)] * 3
    rows = []
    for k in range(3):
        rows.append(tuple(y))                     # stage k input = y_n + h * sum y[j] k_j
        q = [Aw[k] * q[j] + (1 if j == k else 0) for j in range(3)]
        y = [y[j] + Bw[k] * q[j] for j in range(3)]
    A, b, c = omri.kw3_table()
    assert tuple(tuple(r) for r in rows) == tuple(tuple(r) for r in A)
    assert tuple(y) == tuple(b)
    assert tuple(sum(r) for r in A) == tuple(c)


def test_erk_is_third_order_on_closed_forms():
    # y' = -2 y (exp) and y' = y^2 (1/(1-t)): global error ratio 8 per halving
    for f, y0, T, exact in ((lambda y: -2.0 * y, 1.0, 1.0, math.exp(-2.0)),
                            (lambda y: y * y, 0.5, 1.0, 1.0 / (2.0 - 1.0))):
        errs = []
        for n in (20, 40, 80):
            y, h = y0, T / n
            for _ in range(n):
                y = omri.erk_step(f, y, h)
            errs.append(abs(y - exact))
        for e0, e1 in zip(errs, errs[1:]):
            assert 7.0 < e0 / e1 < 9.0


def test_substep_counts():
    # fast step dt/10: intervals of 1/3, 5/12 and 1/4 of dt need 4, 5 and 3 substeps
    assert [omri.substeps(dc, 1e-12, 1e-13) for dc in (1 / 3, 5 / 12, 1 / 4)] == [4, 5, 3]
    assert omri.substeps(0.25, 1.0, 0.25) == 1          # exact fit is not rounded up
    assert omri.substeps(0.25, 1.0, 10.0) == 1


def _mats():
    rng = np.random.default_rng(7)
    AF = rng.standard_normal((3, 3)) * 4.0
    AF = AF - AF.T - 0.5 * np.eye(3)                      # fast, oscillatory
    AS = rng.standard_normal((3, 3)) * 0.7
    return AF, AS


def test_mis_reduces_to_single_rate_methods():
    AF, AS = _mats()
    y0 = np.array([1.0, -0.5, 0.25])
    dt = 0.05
    # no fast part: the slow Knoth-Wolke step
    y1 = omri.mis_step(lambda y: 0.0 * y, lambda y: AS @ y, y0, dt, dt / 7)[0]
    assert np.allclose(y1, omri.erk_step(lambda y: AS @ y, y0, dt), rtol=0, atol=1e-15)
    # no slow part: plain substepping of the fast ODE over the whole step
    y1, _, nf = omri.mis_step(lambda y: AF @ y, lambda y: 0.0 * y, y0, dt, dt / 10)
    ref = y0
    for dc in (1 / 3, 5 / 12, 1 / 4):
        n = omri.substeps(dc, dt, dt / 10)
        for _ in range(n):
            ref = omri.erk_step(lambda y: AF @ y, ref, dc * dt / n)
    assert np.allclose(y1, ref, rtol=0, atol=1e-15)
    assert nf == 36


def test_mis_is_third_order_on_a_split_linear_system():
    # y' = (AF + AS) y with non-commuting parts; exact flow expm; fast
    # substeps fine enough that the slow coupling error dominates
    AF, AS = _mats()
    assert np.abs(AF @ AS - AS @ AF).max() > 1.0
    y0 = np.array([1.0, -0.5, 0.25])
    T = 0.4
    exact = expm((AF + AS) * T) @ y0
    errs = []
    for n in (8, 16, 32):
        y, dt = y0, T / n
        for _ in range(n):
            y = omri.mis_step(lambda u: AF @ u, lambda u: AS @ u, y, dt, dt / 64)[0]
        errs.append(np.abs(y - exact).max())
    orders = [math.log2(e0 / e1) for e0, e1 in zip(errs, errs[1:])]
    assert min(orders) > 2.7, orders


def test_mis_coupling_is_needed_for_third_order():
    # a plausible mistake, forcing every interval with f_S(Y_{i-1}) only,
    # degrades the same system to first order: the pin above would see it
    AF, AS = _mats()
    y0 = np.array([1.0, -0.5, 0.25])
    T = 0.4
    exact = expm((AF + AS) * T) @ y0

    def wrong_step(y, dt):
        for dc in (1 / 3, 5 / 12, 1 / 4):
            r = AS @ y
            n = omri.substeps(dc, dt, dt / 64)
            for _ in range(n):
                y = omri.erk_step(lambda u: AF @ u + r, y, dc * dt / n)
        return y
    errs = []
    for n in (8, 16):
        y = y0
        for _ in range(n):
            y = wrong_step(y, T / n)
        errs.append(np.abs(y - exact).max())
    assert math.log2(errs[0] / errs[1]) < 2.0


GRID = Grid(8, 6, 2, 2e-9, 2e-9, 2e-9)
MAT = dict(Ms=8e5, A=1.3e-11, D=1.5e-3, Ku=3e5, eK=(0.0, 0.0, 1.0), Hbias=(1e4, 0.0, 2e4), alpha=0.1)


def _setup():
    P = tuple(max(2, 1 << (2 * v - 1).bit_length()) for v in (GRID.nz, GRID.ny, GRID.nx))
    spec = onewell.spectrum(GRID, P)
    m0 = random_unit_field((GRID.nx, GRID.ny, GRID.nz), 901, 2)
    return spec, P, m0


def test_llg_split_sums_to_full_rhs():
    spec, P, m0 = _setup()
    p = Params(**MAT, terms=31)
    full = ollg.rhs(GRID, p, m0, spec, P)
    split = omri.fast_rhs(GRID, p, m0) + omri.slow_rhs(GRID, p, m0, spec, P)
    assert np.abs(split - full).max() <= 1e-12 * np.abs(full).max()
    # the fast part is the exchange torque alone: away from the faces (where the
    # DMI boundary condition shapes the ghost cells) it does not see D, Ku,
    # H_bias or demag at all
    q = Params(Ms=MAT["Ms"], A=MAT["A"], alpha=MAT["alpha"], terms=2)
    f_all = omri.fast_rhs(GRID, p, m0)
    f_exch = omri.fast_rhs(GRID, q, m0)
    assert np.array_equal(f_all[:, :, 1:-1, 1:-1], f_exch[:, :, 1:-1, 1:-1])
    assert np.abs(f_all - f_exch).max() > 0


def test_llg_mri_converges_at_third_order_to_the_rk4_solution():
    spec, P, m0 = _setup()
    p = Params(**MAT, terms=31, renorm=0)
    T = 4e-13
    ref = m0.copy()
    for _ in range(400):
        ref = ollg.rk4_step(GRID, p, ref, T / 400, spec, P)
    errs = []
    for n in (4, 8, 16):
        dt = T / n
        m = omri.mri_run(GRID, p, m0, dt, dt / 10, n, spec, P)
        errs.append(np.abs(m - ref).max())
    orders = [math.log2(e0 / e1) for e0, e1 in zip(errs, errs[1:])]
    assert min(orders) > 2.6, (errs, orders)


def test_llg_mri_keeps_unit_length_and_dissipates():
    spec, P, m0 = _setup()
    p = Params(**MAT, terms=31, renorm=2)
    pz = Params(**{**MAT, "Hbias": (0.0, 0.0, 0.0)}, terms=31, renorm=2)
    e0 = ollg.energy(GRID, pz, m0, spec, P)
    m = omri.mri_run(GRID, pz, m0, 2e-13, 2e-14, 5, spec, P)
    assert np.abs(np.sqrt((m * m).sum(0)) - 1.0).max() < 1e-14
    e1 = ollg.energy(GRID, pz, m, spec, P)
    assert e1 < e0
    m1, ns, nf = omri.mri_step(GRID, p, m0, 1e-12, 1e-13, spec, P)
    assert (ns, nf) == (3, 36)
