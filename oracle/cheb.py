"""Chebyshev collocation in the wall-normal direction (oracle; test infrastructure).

Paper: Sec. 2 -- y derivatives are replaced by Chebyshev differentiation
matrices on the Gauss-Lobatto grid, flipped to ascending y (Listing 1); the
fourth derivative inside the bi-Laplacian carries both clamped wall conditions
v = dv/dy = 0 (the Weideman-Reddy weighted interpolant, discussion after
Eq. (Dv_F)); wall rows and columns are truncated to impose homogeneous
Dirichlet conditions (Sec. 3.2, the paragraph after Eq. (CN4)).

All routines are plain FP64 numpy, written from the mathematical definitions.
"""

import numpy as np


def nodes(My):
    """Gauss-Lobatto points in ascending order, y_j = -cos(pi j/(My-1)).

    Listing 1 flips the usual descending Chebyshev grid so that row 0 is the
    lower wall y = -1 and row My-1 is the upper wall y = +1.
    """
    j = np.arange(My)
    return -np.cos(np.pi * j / (My - 1))


def diff_matrix(y):
    """First-derivative collocation matrix on the Chebyshev points ``y``.

    Off-diagonal entries follow the closed form
        D_ij = (c_i / c_j) (-1)^(i+j) / (y_i - y_j),  c = 2 at the two ends,
    which is the derivative of the Lagrange interpolant on these points; the
    diagonal is set so that every row annihilates constants (negative-sum rule).
    The formula is unchanged by reversing the node order.
    """
    My = len(y)
    c = np.ones(My)
    c[0] = 2.0
    c[-1] = 2.0
    c *= (-1.0) ** np.arange(My)
    dy = y[:, None] - y[None, :]
    D = np.outer(c, 1.0 / c) / (dy + np.eye(My))
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, -D.sum(axis=1))
    return D


def dirichlet_d2(D1):
    """Second derivative with homogeneous Dirichlet walls, (D1 D1)[1:-1, 1:-1].

    Sec. 3.2: the inversion matrices for v, eta and W are evaluated with zero
    boundary values by truncating the first and last row and column of the
    differentiation matrix (Listing 1's ``D2F(2:end, 2:end)`` is read as
    ``D2F(2:end-1, 2:end-1)`` so that its size matches ``I = eye(N)``).
    """
    D2 = D1 @ D1
    return D2[1:-1, 1:-1]


def _interior_lagrange_diff(x):
    """Derivative matrix of the Lagrange interpolant on arbitrary points ``x``.

    Barycentric form: with weights w_j = 1 / prod_{k != j} (x_j - x_k),
    D_ij = (w_j / w_i) / (x_i - x_j) for i != j and rows summing to zero.
    """
    n = len(x)
    dx = x[:, None] - x[None, :] + np.eye(n)
    # weights via logarithms would be safer for huge n; n <= 200 here.
    w = 1.0 / np.prod(dx, axis=1)
    D = (w[None, :] / w[:, None]) / dx
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, -D.sum(axis=1))
    return D


def clamped_matrices(My):
    """Clamped derivative operators acting on interior values (Weideman-Reddy).

    A vector of interior values v_j (j = 1..N, N = My - 2) is represented by
        p(y) = sum_j  w(y) l_j(y) / w(y_j) * v_j,   w(y) = (1 - y^2)^2,
    where l_j are the Lagrange polynomials on the N interior nodes.  p vanishes
    with its slope at both walls, i.e. it carries v = dv/dy = 0 (Eq. (b_ve)).
    The m-th derivative of p at the nodes follows from the Leibniz rule,
        D^(m) = [ sum_k C(m,k) diag(w^(m-k)(y_i)) Dt^k ] diag(1 / w(y_j)),
    with Dt the interior Lagrange derivative matrix and
        w' = -4y + 4y^3, w'' = -4 + 12y^2, w''' = 24y, w'''' = 24.

    Returns (D1c, D2c, D4c):
      D1c  (My x N)  first derivative at all nodes (wall rows are exactly 0);
      D2c  (N x N)   second derivative at interior nodes;
      D4c  (N x N)   fourth derivative at interior nodes (the paper's clamped D4).
    """
    y = nodes(My)
    yi = y[1:-1]
    N = My - 2
    Dt = _interior_lagrange_diff(yi)
    Dt2 = Dt @ Dt
    Dt3 = Dt2 @ Dt
    Dt4 = Dt3 @ Dt
    w0 = (1.0 - yi ** 2) ** 2
    w1 = -4.0 * yi + 4.0 * yi ** 3
    w2 = -4.0 + 12.0 * yi ** 2
    w3 = 24.0 * yi
    w4 = 24.0 * np.ones(N)
    S = np.diag(1.0 / w0)
    d = np.diag
    D1c_int = (d(w1) + d(w0) @ Dt) @ S
    D2c = (d(w2) + 2.0 * d(w1) @ Dt + d(w0) @ Dt2) @ S
    D4c = (d(w4) + 4.0 * d(w3) @ Dt + 6.0 * d(w2) @ Dt2
           + 4.0 * d(w1) @ Dt3 + d(w0) @ Dt4) @ S
    D1c = np.zeros((My, N))
    D1c[1:-1, :] = D1c_int
    return D1c, D2c, D4c


def clenshaw_curtis_weights(My):
    """Quadrature weights omega_j with sum_j omega_j f(y_j) = int_{-1}^{1} f dy.

    Defined by exactness on the Chebyshev polynomials T_0..T_{My-1}:
    int T_n = 2 / (1 - n^2) for even n and 0 for odd n.  Solved directly from
    that moment system (the Chebyshev Vandermonde matrix at these points is
    well conditioned).
    """
    y = nodes(My)
    n = np.arange(My)
    V = np.cos(np.outer(n, np.arccos(np.clip(y, -1.0, 1.0))))  # V[n, j] = T_n(y_j)
    moments = np.where(n % 2 == 0, 2.0 / (1.0 - n.astype(float) ** 2 + (n % 2)), 0.0)
    return np.linalg.solve(V, moments)
