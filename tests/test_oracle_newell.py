"""Pins of the oracle's demagnetising tensor against facts the mathematics fixes.

P1 trace, P2 cube self-term, P3 symmetry/parity, P4 near/far agreement and the
dipole limit, P5 an independent surface-charge quadrature, P6 the whole-body
identity for uniformly magnetised boxes.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import newell
from oracle.params import Grid


@pytest.mark.parametrize("d", [(1.0, 1.0, 1.0), (1.3, 0.7, 0.4), (3.90625, 3.90625, 3.0)])
def test_trace_is_one_at_self_and_zero_elsewhere(d):
    # P1: laplacian(1/r) = -4 pi delta  =>  trace N(0) = 1, trace N(R != 0) = 0.
    offs = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (2, 1, 1), (3, 2, 1),
            (5, 0, 2), (7, 3, 1), (12, 9, 4), (30, 2, 1)]
    for o in offs:
        X, Y, Z = (o[0] * d[0], o[1] * d[1], o[2] * d[2])
        t = newell.tensor(X, Y, Z, *d)
        tr = t[0] + t[1] + t[2]
        scale = np.abs(t).max()
        if o == (0, 0, 0):
            assert abs(tr - 1.0) < 1e-13
        else:
            # near-field cancellation grows like eps*(R/d)^6; 1e-9 relative covers
            # cells with 3:1 aspect ratio at r ~ 6
            assert abs(tr) < 1e-9 * scale + 1e-14, (o, tr, scale)


def test_cube_self_term_is_one_third():
    # P2: symmetric cube, trace 1 => each diagonal 1/3, off-diagonals 0.
    t = newell.tensor(0.0, 0.0, 0.0, 2.0, 2.0, 2.0)
    assert np.allclose(t[:3], 1.0 / 3.0, rtol=0, atol=1e-14)
    assert np.allclose(t[3:], 0.0, atol=1e-14)


def test_symmetry_and_parity():
    # P3: diagonals even in every axis; xy odd in x and y, even in z; etc.
    d = (1.1, 0.9, 0.6)
    rng = np.random.default_rng(7)
    for _ in range(20):
        o = rng.integers(0, 15, size=3) * np.array(d)
        base = newell.tensor(*o, *d)
        for sx in (1, -1):
            for sy in (1, -1):
                for sz in (1, -1):
                    t = newell.tensor(sx * o[0], sy * o[1], sz * o[2], *d)
                    for c, name in enumerate(newell.COMPONENTS):
                        px, py, pz = newell.PARITY[name]
                        sgn = (px if sx < 0 else 1) * (py if sy < 0 else 1) * (pz if sz < 0 else 1)
                        assert abs(t[c] - sgn * base[c]) <= 1e-13 * np.abs(base).max() + 1e-300


def test_near_and_far_branches_agree_in_the_overlap():
    # P4: Newell's closed form and the triangle quadrature of the point-dipole
    # kernel are independent derivations of the same integral; where both are
    # accurate (moderate r) they must agree closely.
    # tolerance: rounding in the closed form is amplified ~ (R/d_geo)^6, so
    # cells with a 4:1 aspect ratio get a looser bound
    for d, tol in [((1.0, 1.0, 1.0), 3e-10), ((3.90625, 3.90625, 3.0), 3e-10), ((2.0, 1.0, 0.5), 1e-8)]:
        dm = max(d)
        for o in [(6, 1, 1), (5, 3, 2), (4, 4, 3), (7, 0, 0), (0, 6, 2), (3, 3, 5)]:
            X, Y, Z = (o[0] * d[0], o[1] * d[1], o[2] * d[2])
            r = math.sqrt(X * X + Y * Y + Z * Z) / dm
            if r < 4.5:
                continue
            near = newell.near_tensor(X, Y, Z, *d)
            far = newell.far_tensor(X, Y, Z, *d, 8)[:, 0]
            scale = np.abs(near).max()
            # cancellation in the closed form grows with the cell aspect ratio
            assert np.abs(near - far).max() < tol * scale, (d, o, near, far)


def test_quadrature_converged_for_chosen_orders():
    d = (1.0, 1.0, 1.0)
    for r, q in [(6.0, 6), (12.0, 5), (40.0, 4), (150.0, 3), (2000.0, 2)]:
        for direction in [(1, 0, 0), (1, 1, 0), (1, 1, 1), (0.3, 0.9, 0.2)]:
            u = np.array(direction) / np.linalg.norm(direction) * r
            lo = newell.far_tensor(*u, *d, q)[:, 0]
            hi = newell.far_tensor(*u, *d, 10)[:, 0]
            assert np.abs(lo - hi).max() < 2e-12 * np.abs(hi).max()


def test_dipole_limit():
    # P4: far away, N -> -(V/4pi)(3 RR^T/R^2 - I)/R^3 with O((d/R)^2) correction.
    d = (1.0, 1.0, 1.0)
    for R in [50.0, 200.0, 1000.0]:
        u = np.array([0.6, -0.48, 0.64]) * R
        t = newell.tensor(*u, *d)
        rn = np.linalg.norm(u)
        dip = -(1 / (4 * math.pi)) * (3 * np.outer(u, u) / rn ** 2 - np.eye(3)) / rn ** 3
        ref = np.array([dip[0, 0], dip[1, 1], dip[2, 2], dip[0, 1], dip[0, 2], dip[1, 2]])
        err = np.abs(t - ref).max() / np.abs(ref).max()
        assert err < 2.0 / R ** 2


def _face_pair(h, Y, Z, b, c):
    # Integral of 1/|x-y| over two parallel, equal b x c rectangles whose
    # centres differ by (h, Y, Z) along (normal, u, w): substitute the
    # differences u, w, whose densities are the overlap lengths (b-|u|)(c-|w|).
    def f(w, u):
        r = math.sqrt(h * h + (Y + u) ** 2 + (Z + w) ** 2)
        return (b - abs(u)) * (c - abs(w)) / r if r > 0 else 0.0
    pu = sorted({-Y, 0.0} & {x for x in (-Y, 0.0) if -b < x < b})
    pw = sorted({x for x in (-Z, 0.0) if -c < x < c})
    val, _ = integrate.nquad(f, [[-c, c], [-b, b]],
                             opts=[{"points": pw, "epsabs": 1e-13, "epsrel": 1e-11, "limit": 200},
                                   {"points": pu, "epsabs": 1e-13, "epsrel": 1e-11, "limit": 200}])
    return val


def _surface_nxx(X, Y, Z, dx, dy, dz):
    # N_xx = 1/(4 pi V) sum over the x-faces of both cells of n_x(t) n_x(s) * (face-pair integral),
    # the surface-charge form of the cell-averaged tensor.
    tot = 0.0
    for s in (1, -1):
        for t in (1, -1):
            h = X + t * dx / 2 - s * dx / 2
            tot += s * t * _face_pair(h, Y, Z, dy, dz)
    return tot / (4 * math.pi * dx * dy * dz)


@pytest.mark.parametrize("o", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (2, 0, 0), (1, 1, 1)])
def test_diagonal_matches_independent_surface_integral(o):
    # P5: adaptive quadrature of the surface-charge double integral (no f/g).
    d = (1.2, 1.0, 0.8)
    X, Y, Z = o[0] * d[0], o[1] * d[1], o[2] * d[2]
    ref = _surface_nxx(X, Y, Z, *d)
    got = newell.tensor(X, Y, Z, *d)[0]
    assert abs(got - ref) < 1e-8 * max(abs(ref), 1e-3), (o, got, ref)


def _box_average(n, d, comp):
    # cell-average over a box of cells of sum_j N(r_i - r_j): by additivity of
    # the field, equals the self-term of the whole box.
    nx, ny, nz = n
    I = np.arange(-(nx - 1), nx)
    J = np.arange(-(ny - 1), ny)
    K = np.arange(-(nz - 1), nz)
    kk, jj, ii = np.meshgrid(K, J, I, indexing="ij")
    t = newell.tensor(ii * d[0], jj * d[1], kk * d[2], *d)
    w = (nx - np.abs(ii)) * (ny - np.abs(jj)) * (nz - np.abs(kk))
    return float(np.sum(t[comp] * w)) / (nx * ny * nz)


@pytest.mark.parametrize("n", [(4, 4, 4), (9, 9, 9), (16, 16, 16)])
def test_uniform_cube_of_cells_has_one_third(n):
    # P6: a cube made of cubic cells, uniformly magnetised: <H_d> = -M/3 exactly.
    d = (1.0, 1.0, 1.0)
    for comp in range(3):
        assert abs(_box_average(n, d, comp) - 1.0 / 3.0) < 2e-11
    for comp in range(3, 6):
        assert abs(_box_average(n, d, comp)) < 2e-11


def test_cube_of_flat_cells_has_one_third():
    # P6 with non-cubic cells: 10x10x20 cells of 1 x 1 x 0.5 form a cube.
    d = (1.0, 1.0, 0.5)
    n = (10, 10, 20)
    for comp in range(3):
        assert abs(_box_average(n, d, comp) - 1.0 / 3.0) < 5e-11


def test_box_average_equals_box_self_term():
    # P6 for a flat box: the sum over cell offsets (both branches) equals the
    # closed-form self-term of one big cell of the box's size.
    d = (3.90625, 3.90625, 3.0)
    n = (32, 8, 1)
    box = newell.near_tensor(0.0, 0.0, 0.0, n[0] * d[0], n[1] * d[1], n[2] * d[2])
    for comp in range(6):
        assert abs(_box_average(n, d, comp) - box[comp]) < 5e-11
    # a 125 x 31 x 3 nm film is dominated by N_zz; the full 500 x 125 x 3 nm
    # Standard Problem 4 film is closer to the thin-film limit N_zz -> 1
    assert 0.8 < box[2] < 0.9
    sp4 = newell.near_tensor(0.0, 0.0, 0.0, 500.0, 125.0, 3.0)
    assert 0.95 < sp4[2] < 1.0 and sp4[0] < sp4[1] < 0.05


def test_spectrum_is_real_and_even():
    g = Grid(6, 4, 3, 1.0, 1.2, 0.7)
    spec = newell.spectrum(g)
    assert spec.shape == (6, 6, 8, 7)
    # diagonal spectra are even in ky, kz; real by construction
    for c in range(6):
        sp = spec[c]
        # even or odd in ky and kz like the real-space component
        _, py, pz = newell.PARITY[newell.COMPONENTS[c]]
        flip_y = sp[:, (-np.arange(8)) % 8, :]
        flip_z = sp[(-np.arange(6)) % 6, :, :]
        assert np.allclose(flip_y, py * sp, atol=1e-12)
        assert np.allclose(flip_z, pz * sp, atol=1e-12)


# ---- off-diagonal components, pinned without Newell's g -------------------------------

def _triangle_fold(rho2, zc, c):
    # int_{zc-c}^{zc+c} (c - |w - zc|) / sqrt(rho2 + w^2) dw for rho2 > 0: the
    # shared in-plane direction of two perpendicular faces, whose coordinate
    # difference w has the triangle density (c - |w - zc|) (elementary
    # antiderivatives asinh(w / rho) and sqrt(rho2 + w^2))
    rho = math.sqrt(rho2)
    A = lambda w: math.asinh(w / rho)  # noqa: E731
    B = lambda w: math.sqrt(rho2 + w * w)  # noqa: E731
    lo, hi = zc - c, zc + c
    return ((c - zc) * (A(zc) - A(lo)) + (B(zc) - B(lo))
            + (c + zc) * (A(hi) - A(zc)) - (B(hi) - B(zc)))


def _surface_offdiag(a, b, R, d):
    # N_ab (a != b) = 1/(4 pi V) sum over the a-faces of the target cell (normal
    # sign t) and the b-faces of the source cell (normal sign s) of
    # t s int int dS dS' / |x - x'| -- the surface-charge form of the
    # cell-averaged tensor (Section II-B, Eq. (3)).  The two faces are
    # perpendicular: the difference along a (u) and along b (v) are uniform,
    # the one along the third axis is folded analytically, (u, v) adaptively.
    c = 3 - a - b
    tot = 0.0
    for t in (1, -1):
        for s in (1, -1):
            ua = R[a] + t * d[a] / 2
            vb = R[b] - s * d[b] / 2
            ulo, uhi = ua - d[a] / 2, ua + d[a] / 2
            vlo, vhi = vb - d[b] / 2, vb + d[b] / 2

            def f(v, u):
                r2 = u * u + v * v
                return _triangle_fold(r2, R[c], d[c]) if r2 > 0 else 0.0
            pu = [0.0] if ulo < 0.0 < uhi else []
            pv = [0.0] if vlo < 0.0 < vhi else []
            val, _ = integrate.nquad(f, [[vlo, vhi], [ulo, uhi]],
                                     opts=[{"points": pv, "epsabs": 1e-14, "epsrel": 1e-12, "limit": 200},
                                           {"points": pu, "epsabs": 1e-14, "epsrel": 1e-12, "limit": 200}])
            tot += t * s * val
    return tot / (4 * math.pi * d[0] * d[1] * d[2])


_OFFDIAG = {(0, 1): 3, (0, 2): 4, (1, 2): 5}


@pytest.mark.parametrize("d", [(1.2, 1.0, 0.8), (1.0, 1.0, 1.0), (3.90625, 3.90625, 3.0)])
@pytest.mark.parametrize("o", [(1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1), (2, 1, 0), (1, 2, 1), (2, 2, 1),
                               (-1, 2, 1), (1, -1, -2)])
def test_offdiagonal_matches_independent_surface_integral(o, d):
    # P5 for N_xy, N_xz, N_yz: edge- and corner-touching neighbours and 2-cell
    # offsets, every sign pattern the parity rules of the tensor distinguish.
    # Both orders (a-faces against b-faces and b against a) are evaluated: the
    # tensor is symmetric.
    R = [o[i] * d[i] for i in range(3)]
    got = newell.tensor(*R, *d)
    for (a, b), ci in _OFFDIAG.items():
        ref_ab = _surface_offdiag(a, b, R, d)
        ref_ba = _surface_offdiag(b, a, R, d)
        assert abs(ref_ab - ref_ba) < 1e-12
        assert abs(got[ci] - ref_ab) < 1e-8 * max(abs(ref_ab), 1e-3), (o, (a, b), got[ci], ref_ab)


def _volume_gauss(R, d, nsub=2, q=6):
    # N(R) = -1/(4 pi V) int_target int_source d_a d_b (1/|x - y|) dy dx by a
    # product Gauss-Legendre rule over both cells (nsub panels of q nodes per
    # axis and cell); valid where the cells are apart, so the kernel is smooth
    t, w = np.polynomial.legendre.leggauss(q)
    nodes, wts = [], []
    for i in range(3):
        h = d[i] / nsub
        xs = np.concatenate([-d[i] / 2 + (k + 0.5) * h + 0.5 * h * t for k in range(nsub)])
        nodes.append(xs)
        wts.append(np.tile(0.5 * h * w, nsub))
    X = np.stack(np.meshgrid(*nodes, indexing="ij"), -1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", *wts).ravel()
    acc = np.zeros(6)
    for p in range(X.shape[0]):                      # target node x = R + X[p]
        r = (np.asarray(R) + X[p])[None, :] - X     # x - y for every source node y
        r2 = (r * r).sum(1)
        inv5 = W / (r2 * r2 * np.sqrt(r2))
        K = [(3 * r[:, 0] ** 2 - r2) @ inv5, (3 * r[:, 1] ** 2 - r2) @ inv5, (3 * r[:, 2] ** 2 - r2) @ inv5,
             (3 * r[:, 0] * r[:, 1]) @ inv5, (3 * r[:, 0] * r[:, 2]) @ inv5, (3 * r[:, 1] * r[:, 2]) @ inv5]
        acc += W[p] * np.array(K)
    V = d[0] * d[1] * d[2]
    return -acc / (4 * math.pi * V)


@pytest.mark.slow
@pytest.mark.parametrize("o,d", [((2, 1, 0), (1.0, 1.0, 1.0)), ((2, 1, 1), (1.0, 1.0, 1.0)),
                                 ((0, 2, 1), (1.0, 1.0, 1.0)), ((3, -2, 1), (1.2, 1.0, 0.8)),
                                 ((1, 3, -2), (1.2, 1.0, 0.8)), ((4, 1, 0), (3.90625, 3.90625, 3.0)),
                                 ((2, 2, 2), (1.0, 0.5, 0.75))])
def test_all_components_match_volume_quadrature(o, d):
    # The defining double volume integral of Eq. (3) by brute-force product
    # quadrature (no f, g, triangle densities or near/far split), at offsets
    # where the cells do not touch (r = 2 ... 4.5 cells): every component.
    R = [o[i] * d[i] for i in range(3)]
    got = newell.tensor(*R, *d)
    ref = _volume_gauss(R, d)
    assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max(), (o, d, got, ref)


@pytest.mark.parametrize("o", [(1, 1, 0), (1, 0, 1), (2, 1, 1), (-1, 2, 1), (0, 0, 0)])
def test_tensor_is_additive_over_subcells(o):
    # A 2 x 2 x 2 cell is the union of eight half-size cells: its tensor at
    # offset R is the target-average of the source sum over the subcells,
    # N_big(R) = (1/8) sum_i sum_j N_small(R + s_i - s_j).  Off-centre offsets
    # make all three off-diagonal components non-zero and take the small-cell
    # tensor through every argument pattern of f and g.
    D = (1.2, 1.0, 0.8)
    d = tuple(v / 2 for v in D)
    R = np.array([o[i] * D[i] for i in range(3)])
    subs = [np.array([(i - 0.5) * d[0], (j - 0.5) * d[1], (k - 0.5) * d[2]])
            for i in (0, 1) for j in (0, 1) for k in (0, 1)]
    acc = np.zeros(6)
    for si in subs:
        for sj in subs:
            acc += newell.tensor(*(R + si - sj), *d)
    acc /= 8.0
    big = newell.tensor(*R, *D)
    # rounding of the closed forms' differences: ~1e-15 absolute at these offsets
    assert np.abs(acc - big).max() < 1e-11 * max(np.abs(big).max(), 1e-3), (o, acc, big)
