"""Approximate S3T ensemble (oracle; test infrastructure).

Paper: Sec. 4, the statistical-state-dynamics paragraph -- an ensemble whose
members share one streamwise-mean flow, advanced at every time step by the
perturbation Reynolds stresses averaged over the members, with the perturbations
maintained by stochastic forcing built from eigenvectors of the diffusion
operator acting on a (Lap v, eta) state.  In this module:

* The streamwise mean of a member is its n_x = 0 column (all n_z, plus the
  mean profiles U00, W00); the perturbation is every n_x >= 1 mode.  The shared
  mean is kept identical in every member: at every sub-step the forcing terms of
  the n_x = 0 column (F, G and E_U, E_W) are replaced by their member averages,
  and set_state replaces each member's column by the member average.
* perturbation="linear" (the S3T second-cumulant closure, in which perturbation-
  perturbation advection enters only the mean equation): for n_x >= 1 the
  advection term is U_m . grad u' + u' . grad U_m (U_m = streamwise mean,
  u' = perturbation); for n_x = 0 it is U_m . grad U_m plus the streamwise
  average of u' . grad u'.  perturbation="nonlinear" keeps the full advection.
* Forcing: additive terms f_lapv, f_eta in d(Lap v)/dt and d(eta)/dt, given on
  the interior nodes in the state layout and held constant over a step (the
  RK3 combination weights of every sub-step sum to one, so a constant forcing
  enters each step exactly once).  With the sign conventions of OracleDNS.rhs
  (d Lap v/dt = -F + ..., d eta/dt = -G + ...) this is F -> F - f_lapv,
  G -> G - f_eta.
* frozen_mean=True keeps the streamwise mean fixed (a base flow), so that the
  linear perturbation dynamics are those of the Navier-Stokes equations
  linearised about it (App. B); perturbation="adjoint" advances the adjoint of
  that linearised advection backwards in time: for a velocity lambda' of the
  n_x >= 1 modes the advection term is -(U_m . grad) lambda' + (grad U_m)^T lambda',
  i.e. component j is -U_m . grad lambda'_j + sum_i lambda'_i d_j U_m,i (with the
  mean divergence-free and V_m = 0 at the walls; the viscous and pressure parts
  are self-adjoint, so the same CN operators serve both directions).
"""

import numpy as np

from .step import OracleDNS


class OracleS3T(OracleDNS):
    """Shared-mean ensemble with optional quasi-linear perturbations and forcing."""

    def __init__(self, *args, perturbation="linear", frozen_mean=False, **kw):
        if perturbation not in ("linear", "nonlinear", "adjoint"):
            raise ValueError("perturbation must be 'linear', 'nonlinear' or 'adjoint'")
        self.perturbation = perturbation
        self.frozen_mean = frozen_mean
        super().__init__(*args, **kw)
        if self.advection != "convective":
            raise ValueError("the shared-mean ensemble uses the advective form")
        self.f_lapv = None
        self.f_eta = None

    # ---- state ---------------------------------------------------------------------
    def share(self):
        """Replace every member's streamwise mean by the member average."""
        self.v[:, 0] = self.v[:, 0].mean(axis=0)
        self.eta[:, 0] = self.eta[:, 0].mean(axis=0)
        self.U[:] = self.U.mean(axis=0)
        self.W[:] = self.W.mean(axis=0)

    def set_state(self, v, eta, U, W):
        super().set_state(v, eta, U, W)
        self.share()

    def set_forcing(self, f_lapv=None, f_eta=None):
        self.f_lapv = None if f_lapv is None else np.array(f_lapv, dtype=complex)
        self.f_eta = None if f_eta is None else np.array(f_eta, dtype=complex)

    # ---- advection -------------------------------------------------------------------
    @staticmethod
    def split(vel):
        """(streamwise mean, perturbation) parts of every spectral field."""
        mean, pert = {}, {}
        for k, a in vel.items():
            m = np.zeros_like(a)
            m[..., 0, :] = a[..., 0, :]
            mean[k] = m
            pert[k] = a - m
        return mean, pert

    def advect(self, a, b):
        """Dealiased a . grad b_i (velocity of a, gradients of b), truncated."""
        g = self.grid
        ikx = 1j * g.KX
        ikz = 1j * g.KZ
        P = g.to_physical
        out = [np.zeros_like(b["u"]) for _ in range(3)]
        for e in range(b["u"].shape[0]):
            ua, va, wa = P(a["u"][e]), P(a["v"][e]), P(a["w"][e])
            for i, (f, fy) in enumerate((("u", "uy"), ("v", "vy"), ("w", "wy"))):
                bh = b[f][e]
                n = ua * P(ikx * bh) + va * P(b[fy][e]) + wa * P(ikz * bh)
                out[i][e] = g.to_spectral(n)
        return out

    def transpose_advect(self, a, b):
        """Dealiased component j = sum_i a_i d_j b_i, truncated."""
        g = self.grid
        P = g.to_physical
        out = [np.zeros_like(b["u"]) for _ in range(3)]
        for e in range(b["u"].shape[0]):
            aa = [P(a[f][e]) for f in ("u", "v", "w")]
            for j, d in enumerate(("x", "y", "z")):
                n = 0.0
                for i, f in enumerate(("u", "v", "w")):
                    if d == "x":
                        db = P(1j * g.KX * b[f][e])
                    elif d == "z":
                        db = P(1j * g.KZ * b[f][e])
                    else:
                        db = P(b[f + "y"][e])
                    n = n + aa[i] * db
                out[j][e] = g.to_spectral(n)
        return out

    def nonlinear_adjoint(self, vel):
        """Adjoint of the linearised advection for the n_x >= 1 modes; the
        n_x = 0 column (the frozen base flow's) is zero."""
        m, p = self.split(vel)
        mp = self.advect(m, p)
        tr = self.transpose_advect(p, m)
        out = []
        for i in range(3):
            x = -mp[i] + tr[i]
            x[..., 0, :] = 0.0
            out.append(x)
        uv, wv = self.plane_means(vel)
        return out[0], out[1], out[2], uv, wv

    def plane_means(self, vel):
        P = self.grid.to_physical
        E = vel["u"].shape[0]
        uv = np.zeros((E, self.My))
        wv = np.zeros((E, self.My))
        for e in range(E):
            u, v, w = P(vel["u"][e]), P(vel["v"][e]), P(vel["w"][e])
            uv[e] = (u * v).mean(axis=(-2, -1))
            wv[e] = (w * v).mean(axis=(-2, -1))
        return uv, wv

    def nonlinear_quasilinear(self, vel):
        """Advection with the perturbation-perturbation products kept only in
        the n_x = 0 column; plane means as in the full dynamics."""
        m, p = self.split(vel)
        mm = self.advect(m, m)
        mp = self.advect(m, p)
        pm = self.advect(p, m)
        pp = self.advect(p, p)
        out = []
        for i in range(3):
            ppm = np.zeros_like(pp[i])
            ppm[..., 0, :] = pp[i][..., 0, :]
            out.append(mm[i] + mp[i] + pm[i] + ppm)
        uv, wv = self.plane_means(vel)
        return out[0], out[1], out[2], uv, wv

    # ---- one sub-step's forcing terms -------------------------------------------------
    def stage_terms(self, x):
        vel = self.velocities(*x)
        if self.perturbation == "linear":
            N = self.nonlinear_quasilinear(vel)
        elif self.perturbation == "adjoint":
            N = self.nonlinear_adjoint(vel)
        else:
            N = self.nonlinear(vel)
        F, G, EU, EW = self.rhs(*N)
        if self.f_lapv is not None:
            F = F - self.f_lapv
        if self.f_eta is not None:
            G = G - self.f_eta
        # member averages of the shared column's terms (external forcing included)
        F[:, 0] = F[:, 0].mean(axis=0)
        G[:, 0] = G[:, 0].mean(axis=0)
        EU = np.broadcast_to(EU.mean(axis=0), EU.shape).copy()
        EW = np.broadcast_to(EW.mean(axis=0), EW.shape).copy()
        return F, G, EU, EW

    def solve(self, h, x0, Xc):
        v, eta, U, W = super().solve(h, x0, Xc)
        if self.frozen_mean:
            v[:, 0], eta[:, 0] = x0[0][:, 0], x0[1][:, 0]
            U, W = x0[2].copy(), x0[3].copy()
        return v, eta, U, W
