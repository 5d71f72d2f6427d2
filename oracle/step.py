"""One CN/RK3 time step of the whole ensemble (oracle; test infrastructure).

Paper: Sec. 2 (Eqs. (Dv), (eta), (U00), (W00) and the wall conditions),
Sec. 3.1 (the CN/RK3 scheme: three sub-steps with h = 1/2, 1, 1 and forcing
F^0, 2F^1 - F^0, (F^0 + 4F^1 + F^2)/6, every sub-step restarting from the state
at t) and Sec. 3.2 (pre-inverted operators, u/w recovery from v and eta, the
mean profiles evaluated separately).  Ensemble members are independent
realisations advanced together; here they are simply a leading array axis.
advection="rotational" replaces the advective term u . grad u by omega x u
(same F and G for fields the grid resolves; see nonlinear_rotational).

State layout (also the host layout of the library's state I/O):
  v, eta : complex (E, Nx/2, Nz-1, Ny-2)  -- interior Chebyshev nodes j = 1..Ny-2
  U, W   : real    (E, Ny)                -- mean profiles, walls included
"""

import numpy as np

from .cheb import clenshaw_curtis_weights
from .spectral import SpectralGrid
from .operators import OperatorSet

COUETTE = 0
POISEUILLE = 1


class OracleDNS:
    """Plain FP64 reference of the ensemble step (Sec. 3)."""

    def __init__(self, flow, Re, Lx, Lz, Nx, Ny, Nz, ensemble, dt, Uw=1.0, flux=4.0 / 3.0,
                 advection="convective", v_discretization="clamped"):
        self.flow = COUETTE if flow in (0, "couette") else POISEUILLE
        if advection not in ("convective", "rotational"):
            raise ValueError("advection must be 'convective' or 'rotational'")
        self.advection = advection
        self.Re, self.dt, self.E = float(Re), float(dt), int(ensemble)
        self.Uw = float(Uw)
        self.grid = SpectralGrid(Lx, Lz, Nx, Nz)
        self.My = Ny
        self.N = Ny - 2
        if self.flow == COUETTE:
            self.U_bottom, self.U_top = -self.Uw, self.Uw
        else:
            self.U_bottom, self.U_top = 0.0, 0.0
        self.Q_target = float(flux)
        self.ops = OperatorSet(self.grid, Ny, self.Re, self.dt, self.U_bottom, self.U_top,
                               v_discretization=v_discretization)
        self.ccw = clenshaw_curtis_weights(Ny)
        self.y = self.ops.y
        self._stack_operators()
        self.gamma = np.zeros(self.E)
        self.set_laminar()

    # ---- set-up ---------------------------------------------------------------
    def _stack_operators(self):
        g, N = self.grid, self.N
        self.stacks = {}
        for h in self.ops.h_values:
            st = {k: np.zeros((g.L, g.NZ, N, N)) for k in ("A_v", "B_v", "A_eta", "B_eta")}
            for (ix, iz), op in self.ops.modes[h].items():
                st["A_v"][ix, iz] = op.A_v
                st["B_v"][ix, iz] = op.B_v
                st["A_eta"][ix, iz] = op.A_eta
                st["B_eta"][ix, iz] = op.B_eta
            self.stacks[h] = st

    def laminar_profile(self):
        if self.flow == COUETTE:
            return self.Uw * self.y
        return 1.0 - self.y ** 2

    def set_laminar(self):
        g = self.grid
        self.v = np.zeros((self.E, g.L, g.NZ, self.N), dtype=complex)
        self.eta = np.zeros_like(self.v)
        self.U = np.tile(self.laminar_profile(), (self.E, 1))
        self.W = np.zeros((self.E, self.My))

    def set_state(self, v, eta, U, W):
        self.v = np.array(v, dtype=complex, copy=True)
        self.eta = np.array(eta, dtype=complex, copy=True)
        self.U = np.array(U, dtype=float, copy=True)
        self.W = np.array(W, dtype=float, copy=True)

    def get_state(self):
        return self.v.copy(), self.eta.copy(), self.U.copy(), self.W.copy()

    # ---- field helpers ----------------------------------------------------------
    def _full(self, a):
        """Interior (E, L, NZ, N) -> all nodes (E, My, L, NZ), zero wall values."""
        out = np.zeros((a.shape[0], self.My) + a.shape[1:3], dtype=complex)
        out[:, 1:-1] = np.moveaxis(a, -1, 1)
        return out

    def _ydiff(self, D, f):
        """Apply a y-matrix D (rows x cols) along axis 1 of f (E, cols, L, NZ)."""
        return np.einsum("ij,ejlm->eilm", D, f)

    # ---- a1: velocities and wall-normal gradients (Sec. 3.2, u/w recovery) ------
    def velocities(self, v, eta, U, W):
        """Spectral u, v, w and their y-derivatives at all Chebyshev nodes.

        d_y v = D1c v (clamped representation of v); for k^2 > 0,
          u = (i kx d_y v - i kz eta) / k^2,  w = (i kx eta + i kz d_y v) / k^2;
        the (0,0) mode carries the mean profiles U00 and W00 (v00 = eta00 = 0).
        d_y u = D1 u and d_y w = D1 w on the full grid.
        """
        g = self.grid
        N = self.N
        vint = np.moveaxis(v, -1, 1)                       # (E, N, L, NZ)
        dv = self._ydiff(self.ops.D1c, vint)               # (E, My, L, NZ)
        vf = self._full(v)
        ef = self._full(eta)
        k2 = np.where(g.K2 > 0.0, g.K2, 1.0)
        ikx = 1j * g.KX
        ikz = 1j * g.KZ
        u = (ikx * dv - ikz * ef) / k2
        w = (ikx * ef + ikz * dv) / k2
        u[:, :, 0, 0] = U
        w[:, :, 0, 0] = W
        vf[:, :, 0, 0] = 0.0
        dv[:, :, 0, 0] = 0.0
        uy = self._ydiff(self.ops.D1, u)
        wy = self._ydiff(self.ops.D1, w)
        del N
        return {"u": u, "v": vf, "w": w, "uy": uy, "vy": dv, "wy": wy}

    # ---- a2-a4: de-aliased advection term (Sec. 3.1 and 3.2) --------------------
    def nonlinear(self, vel):
        """N_i = u . grad u_i on the 3/2 grid, forward-transformed and truncated.

        Also returns the plane means <uv>(y) and <wv>(y) that force U00 and W00.
        Members are processed one at a time to bound memory.
        """
        g = self.grid
        ikx = 1j * g.KX
        ikz = 1j * g.KZ
        E = vel["u"].shape[0]
        out_u = np.zeros_like(vel["u"])
        out_v = np.zeros_like(vel["u"])
        out_w = np.zeros_like(vel["u"])
        uv = np.zeros((E, self.My))
        wv = np.zeros((E, self.My))
        for e in range(E):
            P = g.to_physical
            uh, vh, wh = vel["u"][e], vel["v"][e], vel["w"][e]
            u, v, w = P(uh), P(vh), P(wh)
            ux, uy, uz = P(ikx * uh), P(vel["uy"][e]), P(ikz * uh)
            vx, vy, vz = P(ikx * vh), P(vel["vy"][e]), P(ikz * vh)
            wx, wy, wz = P(ikx * wh), P(vel["wy"][e]), P(ikz * wh)
            Nu = u * ux + v * uy + w * uz
            Nv = u * vx + v * vy + w * vz
            Nw = u * wx + v * wy + w * wz
            uv[e] = (u * v).mean(axis=(-2, -1))
            wv[e] = (w * v).mean(axis=(-2, -1))
            out_u[e] = g.to_spectral(Nu)
            out_v[e] = g.to_spectral(Nv)
            out_w[e] = g.to_spectral(Nw)
        return out_u, out_v, out_w, uv, wv

    def nonlinear_rotational(self, vel):
        """Rotational form N = omega x u on the 3/2 grid, forward-transformed and
        truncated; the plane means <uv>, <wv> are those of the advective form.

        The momentum equation (Sec. 2, Eq. (1)) may carry its advection term as
        u . grad u = omega x u + grad(|u|^2 / 2), with the gradient absorbed into
        the pressure.  The v-eta equations take only the curl and the curl of the
        curl of N (F and G below), which annihilate gradients, so this form needs
        u, v, w and the three vorticity components in physical space (6 inverse
        transforms instead of 12):
          omega_x = d_y w - i kz v,  omega_y = i kz u - i kx w,  omega_z = i kx v - d_y u,
          N = (omega_y w - omega_z v, omega_z u - omega_x w, omega_x v - omega_y u).
        """
        g = self.grid
        ikx = 1j * g.KX
        ikz = 1j * g.KZ
        E = vel["u"].shape[0]
        out_u = np.zeros_like(vel["u"])
        out_v = np.zeros_like(vel["u"])
        out_w = np.zeros_like(vel["u"])
        uv = np.zeros((E, self.My))
        wv = np.zeros((E, self.My))
        for e in range(E):
            P = g.to_physical
            uh, vh, wh = vel["u"][e], vel["v"][e], vel["w"][e]
            u, v, w = P(uh), P(vh), P(wh)
            ox = P(vel["wy"][e] - ikz * vh)
            oy = P(ikz * uh - ikx * wh)
            oz = P(ikx * vh - vel["uy"][e])
            uv[e] = (u * v).mean(axis=(-2, -1))
            wv[e] = (w * v).mean(axis=(-2, -1))
            out_u[e] = g.to_spectral(oy * w - oz * v)
            out_v[e] = g.to_spectral(oz * u - ox * w)
            out_w[e] = g.to_spectral(ox * v - oy * u)
        return out_u, out_v, out_w, uv, wv

    # ---- a5: right-hand sides of Eqs. (Dv), (eta), (U00), (W00) -----------------
    def rhs(self, Nu, Nv, Nw, uv, wv):
        """F, G (interior rows) with d_t Lap v = -F + ..., d_t eta = -G + ...;
        E_U = -d_y<uv>, E_W = -d_y<wv> (interior rows)."""
        g = self.grid
        ikx = 1j * g.KX
        ikz = 1j * g.KZ
        D1 = self.ops.D1
        F = -g.K2 * Nv - self._ydiff(D1, ikx * Nu + ikz * Nw)
        G = ikz * Nu - ikx * Nw
        EU = -(uv @ D1.T)
        EW = -(wv @ D1.T)
        F = np.moveaxis(F[:, 1:-1], 1, -1)                 # (E, L, NZ, N)
        G = np.moveaxis(G[:, 1:-1], 1, -1)
        return F, G, EU[:, 1:-1], EW[:, 1:-1]

    # ---- a6-a8: implicit solves (Eqs. (CN1)-(CN4)) ------------------------------
    def solve(self, h, x0, Xc):
        v0, eta0, U0, W0 = x0
        F, G, EU, EW = Xc
        st = self.stacks[h]
        hdt = h * self.dt
        # per (kx, kz): (N x N) @ (N,) for every member -- the ensemble columns
        v = (np.einsum("lmij,elmj->elmi", st["A_v"], v0)
             - hdt * np.einsum("lmij,elmj->elmi", st["B_v"], F))
        eta = (np.einsum("lmij,elmj->elmi", st["A_eta"], eta0)
               - hdt * np.einsum("lmij,elmj->elmi", st["B_eta"], G))
        mo = self.ops.mean[h]
        Uint = U0[:, 1:-1] @ mo.A_U.T + mo.lift + hdt * (EU @ mo.B_U.T)
        Wint = W0[:, 1:-1] @ mo.A_U.T + hdt * (EW @ mo.B_U.T)
        U = np.empty_like(U0)
        U[:, 0], U[:, -1] = self.U_bottom, self.U_top
        U[:, 1:-1] = Uint
        if self.flow == POISEUILLE:
            # gamma(t) holds the bulk flux int U dy at its target (Eq. (U00)):
            # the CN response to gamma is gamma * green, so solve the scalar
            # constraint sum_j w_j U_j = Q exactly at every sub-step.
            q_a = U @ self.ccw
            gamma = (self.Q_target - q_a) / (self.ccw[1:-1] @ mo.green)
            U[:, 1:-1] += gamma[:, None] * mo.green[None, :]
            self.gamma = gamma
        W = np.zeros_like(W0)
        W[:, 1:-1] = Wint
        return v, eta, U, W

    # ---- a10: one full time step --------------------------------------------------
    def stage_terms(self, x):
        vel = self.velocities(*x)
        if self.advection == "rotational":
            Nu, Nv, Nw, uv, wv = self.nonlinear_rotational(vel)
        else:
            Nu, Nv, Nw, uv, wv = self.nonlinear(vel)
        return self.rhs(Nu, Nv, Nw, uv, wv)

    def step(self, nsteps=1):
        for _ in range(nsteps):
            x0 = (self.v, self.eta, self.U, self.W)
            X0 = self.stage_terms(x0)
            x1 = self.solve(0.5, x0, X0)                                  # h = 1/2, F^0
            X1 = self.stage_terms(x1)
            Xc = tuple(2.0 * a - b for a, b in zip(X1, X0))
            x2 = self.solve(1.0, x0, Xc)                                  # h = 1, 2F^1 - F^0
            X2 = self.stage_terms(x2)
            Xc = tuple((a + 4.0 * b + c) / 6.0 for a, b, c in zip(X0, X1, X2))
            v, eta, U, W = self.solve(1.0, x0, Xc)                        # h = 1, (F0+4F1+F2)/6
            self.v = self._project(v)
            self.eta = self._project(eta)
            self.U, self.W = U, W

    def _project(self, a):
        """Hermitian projection of the n_x = 0 column, applied once per step."""
        # a: (E, L, NZ, N) -> the projection acts on the (L, NZ) axes
        t = np.moveaxis(a, -1, 1)                       # (E, N, L, NZ)
        t = self.grid.hermitian_project(t)
        return np.moveaxis(t, 1, -1)
