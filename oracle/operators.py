"""Pre-inverted Crank-Nicolson operators (oracle; test infrastructure).

Paper: Sec. 3.2 "Solution with precalculated inverse matrices", Eqs. (CN1)-(CN4)
and Listings 1 and 3.  For every (kx, kz) pair and sub-step fraction h the
left-hand-side matrix of each CN difference equation is inverted once and
multiplied into the constant right-hand-side matrix, so that a stage update is
two matrix products per field:

  v   (CN1):  [I - c Lap^{-1} LapLap] v_new = [I + c Lap^{-1} LapLap] v_0
                                              - h dt Lap^{-1} F
  eta (CN2):  [I - c Lap] eta_new = [I + c Lap] eta_0 - h dt G
  U00 (CN3):  [I - c D2] U_new = [I + c D2] U_0 + wall terms + h dt (gamma + E_U)
  W00 (CN4):  [I - c D2] W_new = [I + c D2] W_0 + h dt E_W

with c = h dt / (2 Re) (Listing 3's ``g``), Lap = D2_D - k^2 I the Dirichlet
Laplacian (Listing 1) and LapLap = D4c - 2 k^2 D2c + k^4 I the bi-Laplacian with
both clamped wall conditions built into the fourth derivative (Sec. 2).
"""

import numpy as np

from .cheb import nodes, diff_matrix, dirichlet_d2, clamped_matrices


class ModeOperators:
    """A_v, B_v, A_eta, B_eta for one wavenumber pair and one h (folded form).

    v_new   = A_v   v_0   - h dt B_v   F_c
    eta_new = A_eta eta_0 - h dt B_eta G_c
    """

    def __init__(self, D2D, D2c, D4c, k2, c):
        N = D2D.shape[0]
        I = np.eye(N)
        lap = D2D - k2 * I
        laplap = D4c - 2.0 * k2 * D2c + k2 * k2 * I
        # Listing 1: the inverse Laplacian with Dirichlet walls.
        ilap = np.linalg.solve(lap, I)
        # Eq. (CN1): L = Lap^{-1} LapLap; invert [I - c L] and fold it into
        # the constant right-hand-side matrices (Sec. 3.2, preconditioning idea).
        L = ilap @ laplap
        lhs = I - c * L
        self.A_v = np.linalg.solve(lhs, I + c * L)
        self.B_v = np.linalg.solve(lhs, ilap)
        # Eq. (CN2) / Listing 3: ICg = [I - g Lap]^{-1}, ICgCg = ICg [I + g Lap].
        lhs_e = I - c * lap
        self.B_eta = np.linalg.solve(lhs_e, I)
        self.A_eta = self.B_eta @ (I + c * lap)


def kmm_v_operators(D1, D2, k2, c):
    """A_v, B_v of the Helmholtz-Poisson (Kim-Moin-Moser) discretization of
    the v equation: the same CN step (CN1) written for phi = Lap v,

      [I - c Lap] phi_new = [I + c Lap] phi_0 - h dt F     (interior nodes)
      Lap v_new = phi_new                                   (interior nodes)
      v_new = 0, d v_new / dy = 0                           (walls)

    with phi a polynomial on all My nodes (its wall values are the unknowns
    that the influence-matrix method determines) and phi_0 = Lap v_0 on all
    nodes.  Solved here as one block system for (phi, v):
      v_new = A_v v_0 - h dt B_v F.
    Alternative to the clamped fourth-derivative operator of Sec. 2; both are
    spectral discretizations of the same equation and converge to each other."""
    My = D1.shape[0]
    N = My - 2
    lapf = D2 - k2 * np.eye(My)              # full-grid Laplacian
    M = np.zeros((My + N, My + N))
    # Helmholtz rows (interior): phi - c Lap phi
    M[:N, :My] = np.eye(My)[1:-1] - c * lapf[1:-1]
    # Poisson rows (interior): Lap v (v = 0 at the walls) - phi
    M[N:2 * N, My:] = lapf[1:-1, 1:-1]
    M[N:2 * N, :My] = -np.eye(My)[1:-1]
    # clamped walls: d v / dy = 0
    M[2 * N, My:] = D1[0, 1:-1]
    M[2 * N + 1, My:] = D1[-1, 1:-1]
    S = np.linalg.solve(M, np.eye(My + N)[:, :N])[My:]         # v_new per unit R
    # R = [I + c Lap] Lap v_0 on the interior rows
    Q = ((np.eye(My) + c * lapf) @ lapf[:, 1:-1])[1:-1]
    return S @ Q, S


class MeanOperators:
    """Operators for the (kx, kz) = (0, 0) profiles U00 and W00, Eqs. (CN3)-(CN4).

    U_int_new = A_U U_int_0 + lift + h dt B_U E_U,c + gamma * green
    W_int_new = A_U W_int_0 + h dt B_U E_W,c

    ``lift`` carries the wall values: the first and last columns of
    [I - c d_yy] multiply the known wall velocities and are moved to the right-hand
    side (Sec. 3.2, the Couette special case); with CN both time levels
    contribute, giving 2 c D2[int, wall] U_wall.  ``green`` = h dt B_U 1 is the
    response to a unit pressure-gradient forcing, used to hold the bulk flux.
    """

    def __init__(self, D2full, c, hdt, U_bottom, U_top):
        N = D2full.shape[0] - 2
        I = np.eye(N)
        D2D = D2full[1:-1, 1:-1]
        lhs = I - c * D2D
        self.B_U = np.linalg.solve(lhs, I)
        self.A_U = self.B_U @ (I + c * D2D)
        wall_cols = D2full[1:-1, 0] * U_bottom + D2full[1:-1, -1] * U_top
        self.lift = self.B_U @ (2.0 * c * wall_cols)
        self.green = hdt * (self.B_U @ np.ones(N))


class OperatorSet:
    """All operators of one run: Chebyshev matrices and per-h CN operators."""

    def __init__(self, grid, My, Re, dt, U_bottom, U_top, v_discretization="clamped"):
        if v_discretization not in ("clamped", "kmm"):
            raise ValueError("v_discretization must be 'clamped' or 'kmm'")
        self.My = My
        self.N = My - 2
        self.y = nodes(My)
        self.D1 = diff_matrix(self.y)
        self.D2 = self.D1 @ self.D1
        self.D2D = dirichlet_d2(self.D1)
        self.D1c, self.D2c, self.D4c = clamped_matrices(My)
        self.Re = Re
        self.dt = dt
        self.h_values = (0.5, 1.0)
        self.modes = {}
        self.mean = {}
        for h in self.h_values:
            c = h * dt / (2.0 * Re)
            per = {}
            for ix in range(grid.L):
                for iz in range(grid.NZ):
                    k2 = grid.K2[ix, iz]
                    if k2 == 0.0:
                        continue
                    op = ModeOperators(self.D2D, self.D2c, self.D4c, k2, c)
                    if v_discretization == "kmm":
                        op.A_v, op.B_v = kmm_v_operators(self.D1, self.D2, k2, c)
                    per[(ix, iz)] = op
            self.modes[h] = per
            self.mean[h] = MeanOperators(self.D2, c, h * dt, U_bottom, U_top)
