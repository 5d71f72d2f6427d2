"""Pins of the oracle's x-z transforms (CPU).

Paper Sec. 3.2: pseudo-spectral products are de-aliased with the 2/3 rule and
only half of the conjugate harmonic pairs is stored.  Checked against single
Fourier modes, Parseval, and a brute-force convolution on a tiny grid.
"""

import itertools

import numpy as np
import pytest

from oracle.spectral import SpectralGrid


@pytest.fixture(params=[(2 * np.pi, np.pi, 8, 8), (1.75 * np.pi, 1.2 * np.pi, 16, 12)])
def grid(request):
    return SpectralGrid(*request.param)


def hermitian_random(g, rng, shape=()):
    f = rng.standard_normal(shape + (g.L, g.NZ)) + 1j * rng.standard_normal(shape + (g.L, g.NZ))
    f[..., 0, 0] = f[..., 0, 0].real
    return g.hermitian_project(f)


def test_single_mode_is_exact_cosine(grid):
    g = grid
    x, z = g.physical_coords()
    X, Z = np.meshgrid(x, z)            # (Mz, Mx)
    rng = np.random.default_rng(1)
    for ix, iz in [(1, 0), (g.L - 1, 1), (2, g.NZ - 1), (0, 1)]:
        a = complex(rng.standard_normal(), rng.standard_normal())
        fh = np.zeros((g.L, g.NZ), dtype=complex)
        fh[ix, iz] = a
        if ix == 0:
            fh[0, g.conj_iz[iz]] = np.conj(a)
        phase = g.kx[ix] * X + g.kz[iz] * Z
        expect = 2.0 * np.real(a * np.exp(1j * phase))
        np.testing.assert_allclose(g.to_physical(fh), expect, atol=1e-13)


def test_round_trip_and_parseval(grid):
    g = grid
    rng = np.random.default_rng(2)
    fh = hermitian_random(g, rng, (3,))
    f = g.to_physical(fh)
    np.testing.assert_allclose(g.to_spectral(f), fh, atol=1e-14)
    parseval = np.einsum("lm,elm->e", g.mk, np.abs(fh) ** 2)
    np.testing.assert_allclose((f ** 2).mean(axis=(-2, -1)), parseval, rtol=1e-13)


def test_product_matches_bruteforce_convolution():
    """The 3/2 grid makes quadratic products alias-free on the kept modes."""
    g = SpectralGrid(2 * np.pi, 2 * np.pi, 6, 6)     # kept |n| <= 2, 9x9 physical grid
    rng = np.random.default_rng(3)
    ah = hermitian_random(g, rng)
    bh = hermitian_random(g, rng)

    def full(fh):
        d = {}
        for ix, iz in itertools.product(range(g.L), range(g.NZ)):
            nx, nz = int(g.nx[ix]), int(g.nz[iz])
            d[(nx, nz)] = fh[ix, iz]
            if nx > 0:
                d[(-nx, -nz)] = np.conj(fh[ix, iz])
        return d

    A, B = full(ah), full(bh)
    prod = g.to_spectral(g.to_physical(ah) * g.to_physical(bh))
    for ix, iz in itertools.product(range(g.L), range(g.NZ)):
        k = (int(g.nx[ix]), int(g.nz[iz]))
        s = sum(A[p] * B[(k[0] - p[0], k[1] - p[1])] for p in A if (k[0] - p[0], k[1] - p[1]) in B)
        assert abs(prod[ix, iz] - s) <= 1e-13


def test_hermitian_projection_idempotent_and_real_dc(grid):
    g = grid
    rng = np.random.default_rng(4)
    f = rng.standard_normal((g.L, g.NZ)) + 1j * rng.standard_normal((g.L, g.NZ))
    p = g.hermitian_project(f)
    np.testing.assert_allclose(g.hermitian_project(p), p, atol=0)
    assert abs(p[0, 0].imag) < 1e-15
    for iz in range(g.NZ):
        assert abs(p[0, iz] - np.conj(p[0, g.conj_iz[iz]])) < 1e-15
    # the inverse transform only sees the Hermitian part of the n_x = 0 column
    np.testing.assert_allclose(g.to_physical(f), g.to_physical(p), atol=1e-13)
