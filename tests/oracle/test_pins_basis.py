"""Pins of the oracle's B-spline, quadrature, geometry and transfer code
against closed forms and an independent library (scipy.interpolate.BSpline)."""
import numpy as np
import pytest
from scipy.interpolate import BSpline
from scipy import integrate

from oracle import bspline, geometry, hierarchy


def scipy_basis(knots, p, x, der=0):
    n = len(knots) - 1 - p
    out = np.zeros((len(x), n))
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1.0
        s = BSpline(knots, c, p, extrapolate=False)
        out[:, i] = s(x, nu=der) if der else s(x)
    return np.nan_to_num(out)


@pytest.mark.parametrize("p,n_el", [(1, 3), (2, 5), (3, 4), (4, 7), (6, 9)])
def test_partition_of_unity_and_library_values(p, n_el):
    """P1: sum_i B_i = 1, B_i >= 0, sum_i B_i' = 0; values and first two
    derivatives equal scipy's independent B-spline evaluation."""
    rng = np.random.default_rng(p * 100 + n_el)
    x = rng.uniform(0, 1, 200)
    kn = bspline.open_uniform_knots(n_el, p)
    B = bspline.basis_table(kn, p, x)[-1]
    assert B.shape == (200, n_el + p)
    assert np.all(B >= -1e-15)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
    D = bspline.basis_derivative(kn, p, x, 1)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-10)
    np.testing.assert_allclose(B, scipy_basis(kn, p, x), atol=1e-13)
    np.testing.assert_allclose(D, scipy_basis(kn, p, x, 1), atol=1e-10 * n_el)
    if p >= 2:
        D2 = bspline.basis_derivative(kn, p, x, 2)
        np.testing.assert_allclose(D2, scipy_basis(kn, p, x, 2), atol=1e-9 * n_el ** 2)


def test_end_point_values():
    """Open knots interpolate at the ends: B_0(0) = B_{n-1}(1) = 1."""
    kn = bspline.open_uniform_knots(4, 3)
    B = bspline.basis_table(kn, 3, np.array([0.0, 1.0]))[-1]
    np.testing.assert_allclose(B[0], np.eye(7)[0])
    np.testing.assert_allclose(B[1], np.eye(7)[-1])


def test_p1_mass_stiffness_closed_form():
    """P2: p = 1 hat functions: M = h/6 tridiag(1,4,1) (ends 2), K = 1/h tridiag(-1,2,-1) (ends 1)."""
    from oracle.smoothers import mass_stiffness_1d
    n_el = 6
    h = 1.0 / n_el
    M, K = mass_stiffness_1d(n_el, 1)
    n = n_el + 1
    Mr = np.zeros((n, n))
    Kr = np.zeros((n, n))
    for e in range(n_el):
        Mr[e:e + 2, e:e + 2] += h / 6 * np.array([[2, 1], [1, 2]])
        Kr[e:e + 2, e:e + 2] += 1 / h * np.array([[1, -1], [-1, 1]])
    np.testing.assert_allclose(M, Mr, atol=1e-15)
    np.testing.assert_allclose(K, Kr, atol=1e-12)


@pytest.mark.parametrize("p", [2, 3, 5])
def test_mass_stiffness_vs_adaptive_quadrature(p):
    """P2: general p, Gauss tables vs scipy adaptive quadrature of scipy B-splines."""
    from oracle.smoothers import mass_stiffness_1d
    n_el = 4
    kn = bspline.open_uniform_knots(n_el, p)
    M, K = mass_stiffness_1d(n_el, p)
    n = n_el + p
    for i in (0, 1, n // 2):
        for j in range(n):
            ci = np.eye(n)[i]
            cj = np.eye(n)[j]
            si, sj = BSpline(kn, ci, p), BSpline(kn, cj, p)
            di, dj = si.derivative(), sj.derivative()
            brk = list(np.arange(n_el + 1) / n_el)
            m = sum(integrate.quad(lambda t: si(t) * sj(t), a, b)[0] for a, b in zip(brk[:-1], brk[1:]))
            k = sum(integrate.quad(lambda t: di(t) * dj(t), a, b)[0] for a, b in zip(brk[:-1], brk[1:]))
            assert abs(M[i, j] - m) < 1e-12
            assert abs(K[i, j] - k) < 1e-9


def test_gauss_rule_exactness():
    x, w = bspline.gauss_legendre(5)
    for deg in range(10):
        assert abs(np.sum(w * x ** deg) - 1.0 / (deg + 1)) < 1e-15


def test_multilinear_map_jacobian_and_measure():
    """Jacobian equals central finite differences; patch measure equals the
    shoelace area of the quadrilateral (2D) and the unit cube volume (3D)."""
    rng = np.random.default_rng(3)
    c = np.array([[0, 0], [1.2, 0.1], [-0.1, 0.9], [1.1, 1.3]])
    xh = rng.uniform(0, 1, (20, 2))
    X, J = geometry.multilinear(c, xh)
    eps = 1e-6
    for g in range(2):
        e = np.zeros(2)
        e[g] = eps
        Xp, _ = geometry.multilinear(c, xh + e)
        Xm, _ = geometry.multilinear(c, xh - e)
        np.testing.assert_allclose(J[:, :, g], (Xp - Xm) / (2 * eps), atol=1e-8)
    poly = c[[0, 1, 3, 2]]
    area = 0.5 * abs(np.dot(poly[:, 0], np.roll(poly[:, 1], -1)) - np.dot(poly[:, 1], np.roll(poly[:, 0], -1)))
    assert abs(geometry.patch_measure(c) - area) < 1e-14
    cube = np.array([[(b >> 0) & 1, (b >> 1) & 1, (b >> 2) & 1] for b in range(8)], float) * 0.5
    assert abs(geometry.patch_measure(cube) - 0.125) < 1e-15


@pytest.mark.parametrize("p,n_c", [(1, 2), (2, 3), (4, 5), (6, 4)])
def test_prolongation_reproduces_coarse_spline(p, n_c):
    """P4: the coarse spline with coefficients c equals the fine spline with
    coefficients P c at random points (scipy evaluation on both grids)."""
    rng = np.random.default_rng(p + 10 * n_c)
    P = hierarchy.prolongation_1d(n_c, p)
    c = rng.standard_normal(n_c + p)
    kc = bspline.open_uniform_knots(n_c, p)
    kf = bspline.open_uniform_knots(2 * n_c, p)
    x = rng.uniform(0, 1, 300)
    sc = BSpline(kc, c, p)(x)
    sf = BSpline(kf, P @ c, p)(x)
    np.testing.assert_allclose(sf, sc, atol=1e-13)
    # the embedding preserves vanishing boundary values (Dirichlet functions map to Dirichlet functions)
    assert np.all(P[0, 1:] == 0) and np.all(P[-1, :-1] == 0)


def test_level_elements_rule():
    assert [list(e[0]) for e in hierarchy.level_elements([[16, 16]] * 4)] == [[2, 2], [4, 4], [8, 8], [16, 16]]
    lv = hierarchy.level_elements([[64, 64], [96, 96]])
    assert [int(e[0, 0]) for e in lv] == [2, 4, 8, 16, 32, 64]
    assert [int(e[1, 0]) for e in lv] == [3, 6, 12, 24, 48, 96]
    assert int(hierarchy.level_elements([[16, 16]], coarse_min=1)[0][0, 0]) == 1
