"""Pins of the geometry-mask / space-dependent-Ms oracle path.

* A profile equal to 1 everywhere reproduces the uniform field.
* Embedding: a magnet placed inside a larger grid of empty cells has, cell by
  cell, the field and the energy of the same magnet on its own grid (the
  demag tensor is translation invariant and empty cells are sources of
  nothing; the surface of the magnet is a boundary exactly like the faces of
  the small grid).  A plausible mistake in the boundary handling (a missing
  ghost, a wrong normal, an empty neighbour used as m = 0) fails it.
* The demagnetising field of a two-valued Ms equals the direct sum with
  M = Ms(r) m, which shares nothing with the FFT route.
* The local terms scale with 1/Ms of their own cell.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import demag as odemag
from oracle import field as ofield
from oracle import llg as ollg
from oracle import mri as omri
from oracle import newell as onewell
from oracle.params import Grid, Params
from workloads import random_unit_field

MAT = dict(Ms=9e5, A=1.4e-11, D=2.2e-3, Ku=4e5, eK=(0.3, 0.0, 0.95394), Hbias=(1e4, -2e4, 5e3), alpha=0.1)
D3 = (2e-9, 2.5e-9, 1.5e-9)


def _spec(g):
    P = tuple(max(2, 1 << (2 * v - 1).bit_length()) for v in (g.nz, g.ny, g.nx))
    return onewell.spectrum(g, P), P


def test_unit_profile_reproduces_the_uniform_field():
    g = Grid(7, 5, 3, *D3)
    spec, P = _spec(g)
    m = random_unit_field((7, 5, 3), 11, 1)
    p = Params(**MAT, terms=31)
    q = replace(p, ms_profile=np.ones(g.shape))
    a = ofield.heff(g, p, m, spec, P)
    b = ofield.heff(g, q, m, spec, P)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    assert abs(ollg.energy(g, p, m, spec, P) - ollg.energy(g, q, m, spec, P)) <= 1e-12 * abs(
        ollg.energy(g, p, m, spec, P))


@pytest.mark.parametrize("terms", [31, 2 | 4, 1, 8 | 16])
def test_embedded_magnet_has_the_field_of_the_magnet_alone(terms):
    small = Grid(5, 4, 3, *D3)
    big = Grid(9, 7, 5, *D3)
    off = (2, 1, 1)                    # (x, y, z) offset of the magnet in the big grid
    ms_small, P_small = _spec(small)
    ms_big, P_big = _spec(big)
    m_small = random_unit_field((5, 4, 3), 21, 1)
    m_big = random_unit_field((9, 7, 5), 22, 0)      # arbitrary values in the empty cells
    sl = (slice(None), slice(off[2], off[2] + 3), slice(off[1], off[1] + 4), slice(off[0], off[0] + 5))
    m_big[sl] = m_small
    s = np.zeros(big.shape)
    s[sl[1:]] = 1.0
    p = Params(**MAT, terms=terms)
    H_small = ofield.heff(small, p, m_small, ms_small, P_small)
    H_big = ofield.heff(big, replace(p, ms_profile=s), m_big, ms_big, P_big)
    assert np.abs(H_big[sl] - H_small).max() <= 1e-11 * np.abs(H_small).max()
    outside = np.ones(big.shape, dtype=bool)
    outside[sl[1:]] = False
    assert np.all(H_big[:, outside] == 0.0)
    e_small = ollg.energy_parts(small, p, m_small, ms_small, P_small)
    e_big = ollg.energy_parts(big, replace(p, ms_profile=s), m_big, ms_big, P_big)
    for k in e_small:
        assert abs(e_big[k] - e_small[k]) <= 1e-11 * max(abs(e_small["total"]), 1e-30), k


def test_two_valued_ms_demag_matches_the_direct_sum():
    g = Grid(4, 3, 3, 2e-9, 2e-9, 3e-9)
    spec, P = _spec(g)
    m = random_unit_field((4, 3, 3), 31, 0)
    s = np.ones(g.shape)
    s[:, :, 2:] = 0.4
    s[0, 0, 0] = 0.0
    p = Params(Ms=8e5, terms=1, ms_profile=s)
    H = ofield.heff(g, p, m, spec, P)
    Hd = odemag.demag_direct(g, 8e5 * s, m) * (s > 0)[None]
    assert np.abs(H - Hd).max() <= 1e-10 * np.abs(Hd).max()


def test_local_terms_scale_with_the_cell_ms():
    g = Grid(6, 5, 2, *D3)
    m = random_unit_field((6, 5, 2), 41, 1)
    p = Params(**MAT, terms=2 | 4 | 8)
    full = ofield.heff(g, replace(p, ms_profile=np.ones(g.shape)), m)
    half = ofield.heff(g, replace(p, ms_profile=np.full(g.shape, 0.5)), m)
    assert np.abs(half - 2.0 * full).max() <= 1e-12 * np.abs(full).max()


def test_multirate_split_with_a_profile_sums_to_the_full_rhs():
    # the fast (exchange) and slow torques of a masked magnet add up to the
    # full right-hand side of the masked field, and the fast part already
    # honours the magnet's surface (it differs from the unmasked exchange there)
    g = Grid(8, 6, 2, *D3)
    spec, P = _spec(g)
    m = random_unit_field((8, 6, 2), 51, 1)
    s = np.ones(g.shape)
    s[:, :2, :3] = 0.0
    s[:, 4:, :] = 0.5
    p = Params(**MAT, terms=31, ms_profile=s)
    full = ollg.rhs(g, p, m, spec, P)
    split = omri.fast_rhs(g, p, m) + omri.slow_rhs(g, p, m, spec, P)
    assert np.abs(split - full).max() <= 1e-12 * np.abs(full).max()
    plain = omri.fast_rhs(g, replace(p, ms_profile=None), m)
    assert np.abs(omri.fast_rhs(g, p, m) - plain).max() > 1e-3 * np.abs(plain).max()
