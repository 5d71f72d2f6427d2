"""Optimal disturbances by forward-adjoint iteration (oracle; test infrastructure).

Paper: App. B (growth functional G(T) = E(T)/E(0) for perturbations of unit
initial energy density, Navier-Stokes equations linearised about a streamwise-
mean flow, adjoint equations from the Lagrangian) and Sec. 4 (ensemble of
disturbances of one streamwise wavenumber each, iteration of forward and
adjoint integrations over the target time with an orthonormalisation step).

Members of an OracleS3T ensemble with frozen_mean=True hold the base flow in
their n_x = 0 column and one disturbance each in the n_x >= 1 modes.  One
iteration: forward integration over the target time ("linear"), the adjoint
started from the forward end state and integrated over the same time
("adjoint"), then Gram-Schmidt orthonormalisation of the members in the
kinetic-energy inner product, each normalised to energy density 1.  The gains
E(T) of the forward run converge to the leading optimal growths.
"""

import numpy as np

LY = 2.0


def _weights(sim):
    g = sim.grid
    k2 = np.where(g.K2 > 0, g.K2, 1.0)
    mk = g.mk.copy()
    mk[0, :] = 0.0                      # the n_x = 0 column is the base flow
    return k2, mk


def inner(sim, a, b):
    """<a, b> = (1/Ly) int dy sum_k m_k Re(u_a . conj u_b) over the n_x >= 1
    modes of states a = (v, eta), b = (v, eta) (one member each), with
    |u|^2 + |w|^2 = (|dv/dy|^2 + |eta|^2) / k^2 per mode; E = <a, a> / 2."""
    k2, mk = _weights(sim)
    D1c = sim.ops.D1c
    va, ea = a
    vb, eb = b
    dva = np.einsum("jn,lmn->lmj", D1c, va)
    dvb = np.einsum("jn,lmn->lmj", D1c, vb)
    w = sim.ccw
    wi = w[1:-1]
    t = (np.real(va * np.conj(vb)) @ wi + np.real(dva * np.conj(dvb)) @ w / k2
         + np.real(ea * np.conj(eb)) @ wi / k2)
    return float((mk * t).sum() / LY)


def energy(sim, v, eta):
    """Perturbation energy density of every member."""
    return np.array([0.5 * inner(sim, (v[e], eta[e]), (v[e], eta[e])) for e in range(v.shape[0])])


def orthonormalize(sim, v, eta):
    """Modified Gram-Schmidt of the members (in member order) over their n_x >= 1
    modes, each normalised to energy density 1; the n_x = 0 column is kept."""
    v = v.copy()
    eta = eta.copy()
    for i in range(v.shape[0]):
        for j in range(i):
            c = inner(sim, (v[i], eta[i]), (v[j], eta[j])) / 2.0   # <x_j, x_j> = 2
            v[i, 1:] -= c * v[j, 1:]
            eta[i, 1:] -= c * eta[j, 1:]
        n = np.sqrt(0.5 * inner(sim, (v[i], eta[i]), (v[i], eta[i])))
        v[i, 1:] /= n
        eta[i, 1:] /= n
    return v, eta


def optimal_iteration(sim, nsteps, iterations, v0, eta0):
    """Forward-adjoint iterations on a frozen-mean ensemble `sim` (OracleS3T,
    frozen_mean=True) whose current state holds the base flow.  Returns the
    forward gains E(T) of the last iteration and the members' initial states."""
    base_U, base_W = sim.U.copy(), sim.W.copy()
    v, eta = orthonormalize(sim, v0, eta0)
    gains = None
    for _ in range(iterations):
        sim.perturbation = "linear"
        sim.v, sim.eta, sim.U, sim.W = v.copy(), eta.copy(), base_U.copy(), base_W.copy()
        sim.step(nsteps)
        gains = energy(sim, sim.v, sim.eta)
        sim.perturbation = "adjoint"
        sim.step(nsteps)
        v, eta = orthonormalize(sim, sim.v, sim.eta)
    sim.perturbation = "linear"
    return gains, v, eta
