"""Pins of the oracle's demag convolution and local field terms.

P7 FFT convolution = direct O(N^2) sum, P8 padding sufficiency, P9 exchange
eigenvalues, P10 DMI differences and hand-computed edge values, P11 symmetry
of the linear operator K, and energy-gradient identities.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

from oracle import demag, field, newell
from oracle.params import Grid, Params, TERM_DEMAG, TERM_EXCH, TERM_DMI, TERM_ANIS, TERM_ZEEMAN
from workloads import random_unit_field, random_vector_field

MU0 = 4e-7 * math.pi


def _err(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("n", [(5, 3, 2), (8, 8, 1), (7, 5, 3), (4, 4, 4), (1, 1, 1), (9, 1, 1)])
def test_fft_convolution_equals_direct_sum(n):
    # P7: zero padding to twice the size makes the circular convolution the
    # open-boundary linear one.
    g = Grid(*n, 2.0e-9, 1.5e-9, 1.0e-9)
    m = random_unit_field(n, 11)
    H1 = demag.demag_fft(g, 8e5, m)
    H2 = demag.demag_direct(g, 8e5, m)
    assert _err(H1, H2) < 1e-13


def test_padding_three_times_equals_two_times():
    # P8: any extended size >= 2n-1 gives the same convolution.
    n = (6, 5, 3)
    g = Grid(*n, 1e-9, 1e-9, 1e-9)
    m = random_unit_field(n, 12)
    H2 = demag.demag_fft(g, 1e6, m)
    H3 = demag.demag_fft(g, 1e6, m, pshape=(9, 15, 18))
    H11 = demag.demag_fft(g, 1e6, m, pshape=(5, 9, 11))
    assert _err(H3, H2) < 1e-13 and _err(H11, H2) < 1e-13


def test_uniform_cube_demag_average():
    # P6 through the convolution: uniform m in a cube -> <H_d> = -Ms m / 3.
    n = (6, 6, 6)
    g = Grid(*n, 1e-9, 1e-9, 1e-9)
    m = np.zeros((3,) + g.shape)
    m[0] = 0.6
    m[2] = 0.8
    H = demag.demag_fft(g, 1e6, m)
    avg = H.reshape(3, -1).mean(axis=1)
    assert np.allclose(avg, -1e6 / 3 * np.array([0.6, 0.0, 0.8]), rtol=0, atol=1e-8)


def _p(**kw):
    base = dict(Ms=8e5, A=1.3e-11, D=0.0, Ku=0.0, alpha=0.1, terms=TERM_EXCH)
    base.update(kw)
    return Params(**base)


def test_exchange_uniform_is_zero_and_sinusoid_eigenvalue():
    # P9
    n = (16, 3, 2)
    g = Grid(*n, 2e-9, 3e-9, 1e-9)
    p = _p()
    m = np.zeros((3,) + g.shape)
    m[1] = 1.0
    assert np.abs(field.exchange(g, p, m)).max() == 0.0
    k = 2 * math.pi / 7.3e-9
    x = (np.arange(n[0]) + 0.5) * g.dx
    m = np.zeros((3,) + g.shape)
    m[0] = np.cos(k * x)[None, None, :]
    m[1] = np.sin(k * x)[None, None, :]
    H = field.exchange(g, p, m)
    lam = -(4 / g.dx ** 2) * math.sin(k * g.dx / 2) ** 2
    pref = 2 * p.A / (p.mu0 * p.Ms)
    inner = slice(1, -1)
    assert np.allclose(H[:, :, :, inner], pref * lam * m[:, :, :, inner], rtol=1e-12, atol=1e-6)


def test_dmi_linear_field_and_edges():
    # P10: a field linear in x has exact central differences in the interior;
    # uniform m = e_z gives zero in the interior and hand-computed edge values.
    n = (6, 5, 2)
    g = Grid(*n, 2e-9, 2e-9, 2e-9)
    D, A, Ms = 3e-3, 1.6e-11, 1.1e6
    p = _p(D=D, A=A, Ms=Ms, terms=TERM_EXCH | TERM_DMI)
    x = (np.arange(n[0]) + 0.5) * g.dx
    m = np.zeros((3,) + g.shape)
    m[2] = 0.2 + 1e7 * x[None, None, :]
    m[0] = 0.3
    H = field.dmi(g, p, m)
    c = 2 * D / (MU0 * Ms)
    assert np.allclose(H[0][:, 1:-1, 1:-1], c * 1e7, rtol=1e-12)
    assert np.allclose(H[2][:, 1:-1, 1:-1], 0.0, atol=1e-9)
    m = np.zeros((3,) + g.shape)
    m[2] = 1.0
    Hd = field.dmi(g, p, m)
    He = field.exchange(g, p, m)
    assert np.abs(Hd[:, :, 1:-1, 1:-1]).max() == 0.0 and np.abs(He[:, :, 1:-1, 1:-1]).max() == 0.0
    # right x face (outward +x), away from y faces: ghost = m + dx * (-D/2A) * (e_y x e_z)
    # = (dx*kappa, 0, 1):  H_exch,x = -D/(mu0 Ms dx), H_dmi,z = D^2/(2 A mu0 Ms)
    right = (slice(None), slice(1, -1), -1)
    assert np.allclose(He[0][right], -D / (MU0 * Ms * g.dx), rtol=1e-12)
    assert np.allclose(Hd[2][right], D * D / (2 * A * MU0 * Ms), rtol=1e-12)
    assert np.allclose(Hd[0][right], 0.0, atol=1e-9)
    # left x face (outward -x): ghost = (-dx*kappa, 0, 1)
    left = (slice(None), slice(1, -1), 0)
    assert np.allclose(He[0][left], D / (MU0 * Ms * g.dx), rtol=1e-12)
    assert np.allclose(Hd[2][left], D * D / (2 * A * MU0 * Ms), rtol=1e-12)
    # top y face (outward +y): e_z x e_y = -e_x, ghost = m + dy*kappa*(-e_x x e_z) = (0, dy*kappa, 1)
    top = (slice(None), -1, slice(1, -1))
    assert np.allclose(He[1][top], -D / (MU0 * Ms * g.dy), rtol=1e-12)
    assert np.allclose(Hd[2][top], D * D / (2 * A * MU0 * Ms), rtol=1e-12)


@pytest.mark.parametrize("terms", [TERM_EXCH, TERM_EXCH | TERM_DMI, TERM_DEMAG,
                                   TERM_DEMAG | TERM_EXCH | TERM_DMI | TERM_ANIS])
def test_linear_operator_is_symmetric(terms):
    # P11: <u, K v> = <K u, v> (the DMI ghost's skew parts cancel exchange's).
    n = (7, 6, 3)
    g = Grid(*n, 2e-9, 2.5e-9, 1.5e-9)
    p = _p(D=2.5e-3, A=1.6e-11, Ms=1e6, Ku=8e5, eK=(0.36, 0.48, 0.8), terms=terms)
    u = random_vector_field(n, 1)
    v = random_vector_field(n, 2)
    Ku = field.linear_part(g, p, u)
    Kv = field.linear_part(g, p, v)
    a, b = float(np.sum(u * Kv)), float(np.sum(Ku * v))
    assert abs(a - b) <= 1e-13 * np.sqrt(np.sum(Ku * Ku) * np.sum(v * v))


def test_exchange_is_gradient_of_discrete_energy():
    # E = A V sum over neighbour pairs |m_j - m_i|^2 / d^2 (Neumann, D = 0);
    # -1/(mu0 Ms V) dE/dm must equal the exchange field.
    n = (5, 4, 3)
    g = Grid(*n, 2e-9, 3e-9, 1.5e-9)
    p = _p()
    m = random_unit_field(n, 3)
    v = random_vector_field(n, 4)

    def E(mm):
        V = g.volume
        e = 0.0
        for ax, h in ((3, g.dx), (2, g.dy), (1, g.dz)):
            dif = np.diff(mm, axis=ax)
            e += p.A * V * float(np.sum(dif * dif)) / h ** 2
        return e

    eps = 1e-3
    dE = (E(m + eps * v) - E(m - eps * v)) / (2 * eps)
    H = field.exchange(g, p, m)
    ref = -p.mu0 * p.Ms * g.volume * float(np.sum(H * v))
    assert abs(dE - ref) < 1e-10 * abs(ref)


def test_anisotropy_and_demag_are_gradients_of_their_energies():
    n = (4, 3, 2)
    g = Grid(*n, 2e-9, 2e-9, 3e-9)
    p = _p(Ku=5e5, eK=(0.0, 0.6, 0.8), terms=TERM_ANIS | TERM_DEMAG)
    m = random_unit_field(n, 5)
    v = random_vector_field(n, 6)
    eK = np.array(p.eK).reshape(3, 1, 1, 1)

    def Ea(mm):
        return g.volume * p.Ku * float(np.sum(1 - np.sum(eK * mm, axis=0) ** 2))

    def Ed(mm):
        # (mu0 Ms^2 V / 2) sum_ij m_i . N_ij m_j from the direct sum
        Hd = demag.demag_direct(g, p.Ms, mm)
        return -0.5 * p.mu0 * p.Ms * g.volume * float(np.sum(mm * Hd))

    eps = 1e-3
    for Efun, Hfun in ((Ea, lambda mm: field.anisotropy(p, mm)),
                       (Ed, lambda mm: demag.demag_fft(g, p.Ms, mm))):
        dE = (Efun(m + eps * v) - Efun(m - eps * v)) / (2 * eps)
        ref = -p.mu0 * p.Ms * g.volume * float(np.sum(Hfun(m) * v))
        assert abs(dE - ref) < 1e-9 * abs(ref)


def test_dmi_without_exchange_is_rejected():
    g = Grid(3, 3, 1, 1e-9, 1e-9, 1e-9)
    with pytest.raises(ValueError):
        field.heff(g, _p(D=1e-3, terms=TERM_DMI), np.ones((3, 1, 3, 3)))


def test_heff_sums_terms():
    n = (6, 4, 2)
    g = Grid(*n, 2e-9, 2e-9, 2e-9)
    p = _p(D=2e-3, Ku=4e5, Hbias=(1e4, -2e3, 5e3),
           terms=TERM_DEMAG | TERM_EXCH | TERM_DMI | TERM_ANIS | TERM_ZEEMAN)
    m = random_unit_field(n, 9)
    parts = field.heff_parts(g, p, m)
    assert set(parts) == {"demag", "exch", "dmi", "anis", "zeeman"}
    H = field.heff(g, p, m)
    assert np.allclose(H, sum(parts.values()), rtol=0, atol=1e-9)
    Kl = field.linear_part(g, p, m)
    assert np.allclose(H - Kl, np.array(p.Hbias).reshape(3, 1, 1, 1), atol=1e-6)
