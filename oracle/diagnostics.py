"""Diagnostics and one-point statistics (oracle; test infrastructure).

Paper: Sec. 4 -- one-point statistics of the solution: the time-averaged mean
profile U(y), rms fluctuations (u', v', w') about it and the tangential Reynolds
stress u'v'.  Energy, dissipation and power input follow from the
incompressible momentum equation between walls (Sec. 2, Eqs. (1)-(3)):
  dE/dt = Pi - eps,  E = 1/(2V) int |u|^2,  eps = 1/(Re V) int |grad u|^2,
with Pi the work of the moving walls (Couette) or of the pressure gradient
gamma (Poiseuille).  Volume averages use the Clenshaw-Curtis weights over y and
Parseval over the stored half spectrum (weight 1 for n_x = 0, 2 otherwise).
"""

import numpy as np

LY = 2.0


def plane_sq(sim, a, b=None):
    """Plane mean of Re(a conj b) at every node, summed over the stored modes."""
    b = a if b is None else b
    return np.einsum("lm,ejlm->ej", sim.grid.mk, np.real(a * np.conj(b)))


def energy(sim, vel=None):
    """E = 1/(2 Ly) int dy <|u|^2>_xz per member (mean flow included)."""
    vel = sim.velocities(sim.v, sim.eta, sim.U, sim.W) if vel is None else vel
    q = plane_sq(sim, vel["u"]) + plane_sq(sim, vel["v"]) + plane_sq(sim, vel["w"])
    return 0.5 * (q @ sim.ccw) / LY


def dissipation(sim, vel=None):
    """eps = 1/(Re Ly) int dy <sum_ij |d_j u_i|^2>_xz per member."""
    vel = sim.velocities(sim.v, sim.eta, sim.U, sim.W) if vel is None else vel
    g = sim.grid
    tot = 0.0
    for f, fy in (("u", "uy"), ("v", "vy"), ("w", "wy")):
        tot = tot + plane_sq(sim, 1j * g.KX * vel[f]) + plane_sq(sim, vel[fy]) \
            + plane_sq(sim, 1j * g.KZ * vel[f])
    return (tot @ sim.ccw) / (sim.Re * LY)


def dissipation_vorticity(sim, vel=None):
    """eps from the enstrophy: 1/(Re Ly) int dy <|omega|^2>_xz per member.

    For a divergence-free field between no-slip walls (v = 0 and uniform u, w at
    each wall) the volume integrals of |grad u|^2 and |omega|^2 coincide: their
    difference is a divergence whose wall flux u_j d_j v vanishes."""
    vel = sim.velocities(sim.v, sim.eta, sim.U, sim.W) if vel is None else vel
    g = sim.grid
    ox = vel["wy"] - 1j * g.KZ * vel["v"]
    oy = 1j * g.KZ * vel["u"] - 1j * g.KX * vel["w"]
    oz = 1j * g.KX * vel["v"] - vel["uy"]
    tot = plane_sq(sim, ox) + plane_sq(sim, oy) + plane_sq(sim, oz)
    return (tot @ sim.ccw) / (sim.Re * LY)


def wall_shear(sim):
    """dU/dy at the lower and upper wall per member."""
    dU = sim.U @ sim.ops.D1.T
    return dU[:, 0], dU[:, -1]


def power_input(sim):
    """Pi: wall work U_w (U'(1) + U'(-1)) / (Re Ly) for Couette, gamma Q / Ly
    for the constant-flux channel."""
    if sim.flow == 0:
        lo, hi = wall_shear(sim)
        return sim.Uw * (hi + lo) / (sim.Re * LY)
    return sim.gamma * flux(sim) / LY


def flux(sim):
    """Bulk flux Q = int_{-1}^{1} U dy per member."""
    return sim.U @ sim.ccw


def divergence_max(sim, vel=None):
    """max |i kx u + d_y v + i kz w| over modes and nodes, per member."""
    vel = sim.velocities(sim.v, sim.eta, sim.U, sim.W) if vel is None else vel
    g = sim.grid
    div = 1j * g.KX * vel["u"] + vel["vy"] + 1j * g.KZ * vel["w"]
    return np.abs(div).reshape(div.shape[0], -1).max(axis=1)


def profiles(sim, vel=None):
    """Per-member plane quantities used by the one-point statistics.

    Returns a dict of (E, Ny) arrays: mean profiles U00, W00 and the
    fluctuation sums  sum_{k != 0} m_k |u_k|^2 (and v, w) and
    sum_{k != 0} m_k Re(u_k conj v_k).
    """
    vel = sim.velocities(sim.v, sim.eta, sim.U, sim.W) if vel is None else vel
    mask = sim.grid.mk.copy()
    mask[0, 0] = 0.0

    def s(a, b=None):
        b = a if b is None else b
        return np.einsum("lm,ejlm->ej", mask, np.real(a * np.conj(b)))

    return {
        "U": sim.U.copy(), "W": sim.W.copy(),
        "uu": s(vel["u"]), "vv": s(vel["v"]), "ww": s(vel["w"]),
        "uv": s(vel["u"], vel["v"]),
    }


class StatsAccumulator:
    """Time- and ensemble-averaged one-point statistics (Sec. 4).

    Fluctuations are taken about the ensemble- and time-averaged mean U(y):
      u'^2(y) = < sum_{k!=0} m_k |u_k|^2 + (U00 - U)^2 >,  u'v' = < sum m_k Re(u_k v_k*) >.
    """

    def __init__(self):
        self.n = 0
        self.sums = {}

    def add(self, sim):
        p = profiles(sim)
        lo, hi = wall_shear(sim)
        p["U2"] = p["U"] ** 2
        p["W2"] = p["W"] ** 2
        p["dUlo"] = lo
        p["dUhi"] = hi
        for k, val in p.items():
            self.sums[k] = self.sums.get(k, 0.0) + val
        self.n += 1

    def result(self, sim):
        m = {k: v / self.n for k, v in self.sums.items()}
        U = m["U"].mean(axis=0)
        W = m["W"].mean(axis=0)
        U2 = m["U2"].mean(axis=0)
        W2 = m["W2"].mean(axis=0)
        out = {
            "U": U, "W": W,
            "urms": np.sqrt(np.maximum(m["uu"].mean(axis=0) + U2 - U ** 2, 0.0)),
            "vrms": np.sqrt(np.maximum(m["vv"].mean(axis=0), 0.0)),
            "wrms": np.sqrt(np.maximum(m["ww"].mean(axis=0) + W2 - W ** 2, 0.0)),
            "uv": m["uv"].mean(axis=0),
        }
        lo = m["dUlo"].mean()
        hi = m["dUhi"].mean()
        if sim.flow == 0:
            tau = 0.5 * (abs(lo) + abs(hi)) / sim.Re
        else:
            tau = (lo - hi) / (2.0 * sim.Re)
        out["tau_w"] = tau
        out["Re_tau"] = sim.Re * np.sqrt(abs(tau))
        return out
