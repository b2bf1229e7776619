"""Pins of the oracle's LLG right-hand side, renormalisation and RK4.

P12 geometry of the right-hand side and conservation of |m|, P13 the
macrospin closed form and fourth-order convergence, P14 energy decay under
damping, and the paper's printed RK4 stability limit (Table II).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import llg, newell, field
from oracle.params import Grid, Params, TERM_DEMAG, TERM_EXCH, TERM_DMI, TERM_ANIS, TERM_ZEEMAN
from workloads import random_unit_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _params(**kw):
    base = dict(Ms=1e6, A=1.6e-11, D=2.5e-3, Ku=8e5, alpha=0.1, Hbias=(3e4, -1e4, 2e4),
                terms=TERM_DEMAG | TERM_EXCH | TERM_DMI | TERM_ANIS | TERM_ZEEMAN)
    base.update(kw)
    return Params(**base)


def test_rhs_is_tangent():
    # P12: m . R(m) = 0 cell by cell.
    n = (6, 5, 2)
    g = Grid(*n, 2e-9, 2e-9, 2e-9)
    p = _params()
    m = random_unit_field(n, 21)
    R = llg.rhs(g, p, m)
    rel = np.abs(np.sum(m * R, axis=0)).max() / np.abs(R).max()
    assert rel < 1e-15


def test_norm_conservation_by_mode():
    # P12: without renormalisation |m|-1 drifts at O(dt^5) per step (32x per
    # halving of dt); with stage renormalisation |m| = 1 to rounding.
    n = (6, 5, 2)
    g = Grid(*n, 2e-9, 2e-9, 2e-9)
    m0 = random_unit_field(n, 22, smooth=1)
    drift = []
    for dt in (2e-14, 1e-14):
        p = _params(renorm=0)
        m = llg.rk4_step(g, p, m0, dt)
        drift.append(np.abs(np.sqrt(np.sum(m * m, axis=0)) - 1).max())
    assert 20 < drift[0] / drift[1] < 50
    p = _params(renorm=2)
    m = m0
    for _ in range(5):
        m = llg.rk4_step(g, p, m, 2e-14)
    assert np.abs(np.sqrt(np.sum(m * m, axis=0)) - 1).max() < 4e-16


@pytest.mark.parametrize("renorm", [0, 1, 2])
def test_macrospin_closed_form_and_order(renorm):
    # P13: one cubic cell in a field along +z; its self-demag is parallel to m
    # so exerts no torque.  tan(theta/2) decays as exp(-alpha |gamma_L| mu0 H t)
    # and phi advances as |gamma_L| mu0 H t (counter-clockwise about +z).
    g = Grid(1, 1, 1, 2e-9, 2e-9, 2e-9)
    H = 2e5
    p = Params(Ms=8e5, alpha=0.1, Hbias=(0, 0, H), terms=TERM_DEMAG | TERM_ZEEMAN, renorm=renorm)
    th0, ph0, T = 1.0, 0.3, 2e-11
    a = abs(p.mu0 * p.gamma / (1 + p.alpha ** 2))
    th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-p.alpha * a * H * T))
    ph = ph0 + a * H * T
    exact = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    spec = newell.spectrum(g)
    errs = []
    for n in (50, 100, 200):
        m = np.array([math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0),
                      math.cos(th0)]).reshape(3, 1, 1, 1)
        for _ in range(n):
            m = llg.rk4_step(g, p, m, T / n, spec)
        errs.append(np.linalg.norm(m.ravel() - exact))
    assert errs[-1] < 1e-11
    for e0, e1 in zip(errs, errs[1:]):
        assert 14 < e0 / e1 < 18


def test_two_renormalisation_readings_differ_at_fifth_order():
    n = (5, 4, 2)
    g = Grid(*n, 2e-9, 2e-9, 2e-9)
    m0 = random_unit_field(n, 23, smooth=2)
    d = []
    for dt in (4e-14, 2e-14):
        a = llg.rk4_step(g, _params(renorm=1), m0, dt)
        b = llg.rk4_step(g, _params(renorm=2), m0, dt)
        d.append(np.abs(a - b).max())
    assert 25 < d[0] / d[1] < 40


def test_energy_decays_under_damping():
    # P14: with alpha > 0 and a static field, dE/dt = mu0 Ms V a alpha sum |m x H|^2 <= 0.
    n = (16, 8, 1)
    g = Grid(*n, 3.90625e-9, 3.90625e-9, 3e-9)
    p = Params(Ms=8e5, A=1.3e-11, alpha=0.02, Hbias=(19894.37, 0, 0),
               terms=TERM_DEMAG | TERM_EXCH | TERM_ZEEMAN)
    spec = newell.spectrum(g)
    m = random_unit_field(n, 24, smooth=3)
    E = [llg.energy(g, p, m, spec)]
    for _ in range(20):
        m = llg.rk4_step(g, p, m, 1e-13, spec)
        E.append(llg.energy(g, p, m, spec))
    assert all(e1 <= e0 for e0, e1 in zip(E, E[1:]))
    # instantaneous rate matches mu0 Ms V a alpha sum |m x H|^2
    H = field.heff(g, p, m, spec)
    mxH = llg.cross(m, H)
    rate = p.mu0 * p.Ms * g.volume * llg.prefactor(p) * p.alpha * float(np.sum(mxH * mxH))
    dt = 1e-16
    m1 = llg.rk4_step(g, p, m, dt, spec)
    m0 = llg.rk4_step(g, p, m, -dt, spec)
    fd = (llg.energy(g, p, m1, spec) - llg.energy(g, p, m0, spec)) / (2 * dt)
    assert abs(fd - rate) < 1e-6 * abs(rate)


def test_energy_parts_sum_and_uniform_cube_value():
    n = (5, 5, 5)
    g = Grid(*n, 2e-9, 2e-9, 2e-9)
    p = Params(Ms=8e5, A=1.3e-11, terms=TERM_DEMAG | TERM_EXCH)
    m = np.zeros((3,) + g.shape)
    m[1] = 1.0
    e = llg.energy_parts(g, p, m)
    Km = 0.5 * p.mu0 * p.Ms ** 2
    # uniform cube: e_demag / K_m = 1/3, no exchange energy
    assert abs(e["demag"] / (Km * g.volume * g.ncell) - 1 / 3) < 1e-12
    assert abs(e["exch"]) < 1e-30
    q = _params()
    m = random_unit_field(n, 25)
    parts = llg.energy_parts(g, q, m)
    assert abs(parts["total"] - llg.energy(g, q, m)) < 1e-12 * abs(parts["total"])


def test_table2_rk4_stability_limit():
    gold = json.load(open(os.path.join(GOLDEN, "table2_rk4_stability.json")))
    h = gold["cell_m"]
    n = (32, 8, gold["nz"])
    g = Grid(*n, h, h, h)
    mat = gold["material"]
    p = Params(Ms=mat["Ms"], A=mat["A"], alpha=mat["alpha"], terms=TERM_DEMAG | TERM_EXCH)
    spec = newell.spectrum(g)
    m0 = random_unit_field(n, 5, smooth=3)
    E0 = llg.energy(g, p, m0, spec)
    res = {}
    for dt in (gold["rk4_max_stable_dt_s"], 2 * gold["rk4_max_stable_dt_s"]):
        m = m0
        for _ in range(40):
            m = llg.rk4_step(g, p, m, dt, spec)
        res[dt] = llg.energy(g, p, m, spec) / E0
    stable, unstable = res[gold["rk4_max_stable_dt_s"]], res[2 * gold["rk4_max_stable_dt_s"]]
    assert stable < 1.0
    assert unstable > 1.2
