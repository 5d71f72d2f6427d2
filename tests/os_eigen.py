"""Orr-Sommerfeld eigenvalue solver used to pin the oracle's v operator.

Independent of the time stepper: it discretises the linear stability problem
of plane Poiseuille flow directly as a generalised eigenproblem,
    [LapLap/Re - i a U Lap + i a U''] phi = lam Lap phi,   lam = -i a c,
with the same Chebyshev matrices (Dirichlet Lap, clamped LapLap) that the paper
uses for the v equation (Sec. 2).  Orszag (1971) gives the least-stable mode at
Re = 10^4, a = 1 as c = 0.23752649 + 0.00373967 i.
"""

import numpy as np
import scipy.linalg

from oracle.cheb import nodes, diff_matrix, dirichlet_d2, clamped_matrices


def os_modes(Re, alpha, My):
    y = nodes(My)
    yi = y[1:-1]
    D1 = diff_matrix(y)
    D2D = dirichlet_d2(D1)
    _, D2c, D4c = clamped_matrices(My)
    N = My - 2
    I = np.eye(N)
    a2 = alpha * alpha
    lap = D2D - a2 * I
    laplap = D4c - 2.0 * a2 * D2c + a2 * a2 * I
    U = 1.0 - yi ** 2
    Upp = -2.0 * np.ones(N)
    A = laplap / Re - 1j * alpha * np.diag(U) @ lap + 1j * alpha * np.diag(Upp)
    lam, vec = scipy.linalg.eig(A, lap)
    ok = np.isfinite(lam)
    lam, vec = lam[ok], vec[:, ok]
    order = np.argsort(-lam.real)
    lam, vec = lam[order], vec[:, order]
    c = 1j * lam / alpha
    return c, vec
