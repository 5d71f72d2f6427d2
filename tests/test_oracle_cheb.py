"""Pins of the oracle's Chebyshev operators against closed forms (CPU).

Paper Sec. 2: y derivatives are Chebyshev collocation matrices; the fourth
derivative carries the clamped conditions v = v' = 0 (Weideman-Reddy).  Each
matrix must differentiate exactly the polynomial space it represents.
"""

import numpy as np
import numpy.polynomial.polynomial as Poly
import pytest

from oracle import cheb

pytestmark = pytest.mark.parametrize("My", [9, 33, 49, 97])


def test_nodes_ascending_and_symmetric(My):
    y = cheb.nodes(My)
    assert y[0] == -1.0 and y[-1] == 1.0
    assert np.all(np.diff(y) > 0)
    np.testing.assert_allclose(y, -y[::-1], atol=1e-15)


def test_d1_d2_exact_on_monomials(My):
    y = cheb.nodes(My)
    D1 = cheb.diff_matrix(y)
    D2 = D1 @ D1
    for p in range(My):
        c = np.zeros(p + 1)
        c[p] = 1.0
        f = Poly.polyval(y, c)
        d1 = Poly.polyval(y, Poly.polyder(c))
        d2 = Poly.polyval(y, Poly.polyder(c, 2))
        assert np.max(np.abs(D1 @ f - d1)) <= 1e-12 * max(1.0, np.max(np.abs(d1))) * My
        assert np.max(np.abs(D2 @ f - d2)) <= 1e-12 * max(1.0, np.max(np.abs(d2))) * My ** 2


def test_d1_annihilates_constants_and_matches_order(My):
    y = cheb.nodes(My)
    D1 = cheb.diff_matrix(y)
    np.testing.assert_allclose(D1 @ np.ones(My), 0.0, atol=1e-12 * My ** 2)
    # corner entry of the ascending grid: -(2 n^2 + 1)/6 with n = My - 1
    n = My - 1
    np.testing.assert_allclose(D1[0, 0], -(2 * n * n + 1) / 6.0, rtol=1e-12)
    np.testing.assert_allclose(D1[-1, -1], (2 * n * n + 1) / 6.0, rtol=1e-12)


def test_dirichlet_d2_exact_on_wall_vanishing_polynomials(My):
    y = cheb.nodes(My)
    D2D = cheb.dirichlet_d2(cheb.diff_matrix(y))
    yi = y[1:-1]
    for p in range(My - 2):
        c = Poly.polymul([1.0, 0.0, -1.0], np.eye(p + 1)[p])       # (1 - y^2) y^p
        f = Poly.polyval(yi, c)
        d2 = Poly.polyval(yi, Poly.polyder(c, 2))
        assert np.max(np.abs(D2D @ f - d2)) <= 1e-11 * max(1.0, np.max(np.abs(d2))) * My


def test_clamped_operators_exact_on_clamped_polynomials(My):
    """D1c, D2c, D4c differentiate (1 - y^2)^2 p(y), deg p <= N - 1, exactly.

    D4c has entries ~ N^8, so its error is measured normwise relative to
    ||D4c|| ||f||, the scale at which any FP64 representation rounds.
    """
    y = cheb.nodes(My)
    yi = y[1:-1]
    N = My - 2
    D1c, D2c, D4c = cheb.clamped_matrices(My)
    assert D1c.shape == (My, N) and D2c.shape == (N, N) and D4c.shape == (N, N)
    np.testing.assert_array_equal(D1c[0], 0.0)
    np.testing.assert_array_equal(D1c[-1], 0.0)
    n4 = np.max(np.abs(D4c).sum(axis=1))
    n2 = np.max(np.abs(D2c).sum(axis=1))
    n1 = np.max(np.abs(D1c).sum(axis=1))
    rng = np.random.default_rng(7)
    for p in list(range(min(N, 6))) + [N - 1]:
        q = rng.standard_normal(p + 1)
        c = Poly.polymul([1.0, 0.0, -2.0, 0.0, 1.0], q)               # (1-y^2)^2 q(y)
        f = Poly.polyval(yi, c)
        fn = np.max(np.abs(f))
        e1 = np.max(np.abs(D1c @ f - Poly.polyval(y, Poly.polyder(c))))
        e2 = np.max(np.abs(D2c @ f - Poly.polyval(yi, Poly.polyder(c, 2))))
        e4 = np.max(np.abs(D4c @ f - Poly.polyval(yi, Poly.polyder(c, 4))))
        assert e1 <= 1e-13 * n1 * fn * My
        assert e2 <= 1e-13 * n2 * fn * My
        assert e4 <= 1e-13 * n4 * fn * My


def test_clamped_minus_dirichlet_is_rank_two_in_wall_slopes(My):
    """D4c - (D2 D2)[int,int] and D2c - D2D have rank 2, their rows spanned by
    the two wall-slope rows of D1 (restricted to interior columns)."""
    if My < 9:
        pytest.skip("needs a few interior points")
    y = cheb.nodes(My)
    D1 = cheb.diff_matrix(y)
    D2 = D1 @ D1
    D4D = (D2 @ D2)[1:-1, 1:-1]
    _, D2c, D4c = cheb.clamped_matrices(My)
    S = D1[[0, -1], 1:-1]
    for diff in (D4c - D4D, D2c - cheb.dirichlet_d2(D1)):
        coef, *_ = np.linalg.lstsq(S.T, diff.T, rcond=None)
        resid = diff.T - S.T @ coef
        assert np.max(np.abs(resid)) <= 1e-13 * np.max(np.abs(diff)) * My


def test_clenshaw_curtis_integrates_polynomials(My):
    y = cheb.nodes(My)
    w = cheb.clenshaw_curtis_weights(My)
    for p in range(My):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(w @ y ** p - exact) <= 1e-13 * My
    # and a smooth non-polynomial: int cos(pi y / 2) dy = 4 / pi
    if My >= 33:
        assert abs(w @ np.cos(np.pi * y / 2) - 4.0 / np.pi) <= 1e-14
