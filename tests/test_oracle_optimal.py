"""Pins of the optimal-disturbance oracle (CPU).

  * a frozen mean stays bitwise fixed while perturbations evolve;
  * the forward dynamics about a frozen mean are linear in the perturbation;
  * the adjoint advection satisfies <lambda, N_lin u> = <N_adj lambda, u> exactly
    (to round-off) for fields the grid resolves, since it follows from
    integration by parts with a divergence-free mean that vanishes in y at the
    walls (checked on a base flow with rolls and streaks);
  * Gram-Schmidt returns members of unit energy, mutually orthogonal;
  * forward-adjoint iteration converges to sigma_max^2 of the forward
    propagator in the energy norm, assembled column by column on a small grid
    (non-normal transient growth on laminar Couette flow).
"""

import numpy as np

from oracle import OracleS3T
from oracle import optimal as opt
from paper_2306_12739_amd import inputs

BOX = (0, 500.0, 2.0 * np.pi, np.pi, 8, 17, 8)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make(E, box=BOX, dt=0.1, pert="linear"):
    flow, Re, Lx, Lz, Nx, Ny, Nz = box
    sim = OracleS3T(flow, Re, Lx, Lz, Nx, Ny, Nz, E, dt, perturbation=pert, frozen_mean=True)
    sim.set_laminar()
    return sim


def base_with_streaks(box, seed):
    """A state whose n_x = 0 column carries a y-z base flow (rolls and streaks)."""
    flow, Re, Lx, Lz, Nx, Ny, Nz = box
    v, eta, U, W = inputs.random_state(flow, Lx, Lz, Nx, Ny, Nz, 1, 0.3, seed, spectrum="low")
    y = -np.cos(np.pi * np.arange(Ny) / (Ny - 1))
    v[:, 1:] = 0.0
    eta[:, 1:] = 0.0
    U = U + 0.1 * (1 - y ** 2)[None]
    W = W + 0.05 * (1 - y ** 2)[None] * y[None]
    return v, eta, U, W


def test_frozen_mean_and_forward_linearity():
    box = (0, 400.0, 1.75 * np.pi, 1.2 * np.pi, 16, 25, 12)
    bv, be, bU, bW = base_with_streaks(box, 3)
    pv, pe, _, _ = inputs.random_state(0, box[2], box[3], 16, 25, 12, 2, 0.2, 4, spectrum="k2")
    pv[:, 0] = 0.0
    pe[:, 0] = 0.0
    finals = []
    for alpha in (1.0, 0.5):
        sim = OracleS3T(*box, 2, 0.02, perturbation="linear", frozen_mean=True)
        sim.set_state(pv * alpha + bv, pe * alpha + be, np.repeat(bU, 2, 0), np.repeat(bW, 2, 0))
        sim.step(4)
        for e in range(2):
            assert np.array_equal(sim.v[e, 0], bv[0, 0]) and np.array_equal(sim.eta[e, 0], be[0, 0])
            assert np.array_equal(sim.U[e], bU[0]) and np.array_equal(sim.W[e], bW[0])
        finals.append((sim.v[:, 1:].copy(), sim.eta[:, 1:].copy()))
    assert rel(finals[1][0], 0.5 * finals[0][0]) < 1e-13
    assert rel(finals[1][1], 0.5 * finals[0][1]) < 1e-13


def test_adjoint_identity_for_resolved_fields():
    box = (0, 400.0, 1.75 * np.pi, 1.2 * np.pi, 16, 33, 16)
    sim = make(1, box=box)
    bv, be, bU, bW = base_with_streaks(box, 5)
    lv, le, _, _ = inputs.random_state(0, box[2], box[3], 16, 33, 16, 1, 0.2, 6, spectrum="low")
    uv, ue, _, _ = inputs.random_state(0, box[2], box[3], 16, 33, 16, 1, 0.2, 7, spectrum="low")
    for a in (lv, le, uv, ue):
        a[:, 0] = 0.0
    vel_l = sim.velocities(lv + bv, le + be, bU, bW)
    vel_u = sim.velocities(uv + bv, ue + be, bU, bW)
    m, pl = OracleS3T.split(vel_l)
    _, pu = OracleS3T.split(vel_u)
    n_lin = [a + b for a, b in zip(sim.advect(m, pu), sim.advect(pu, m))]
    n_adj = [-a + b for a, b in zip(sim.advect(m, pl), sim.transpose_advect(pl, m))]

    def vel_inner(a, b):
        mk = sim.grid.mk.copy()
        mk[0] = 0.0
        t = sum(np.real(x * np.conj(y)).transpose(0, 2, 3, 1) @ sim.ccw for x, y in zip(a, b))
        return float((mk * t[0]).sum())
    lhs = vel_inner([pl["u"], pl["v"], pl["w"]], n_lin)
    rhs = vel_inner(n_adj, [pu["u"], pu["v"], pu["w"]])
    scale = abs(vel_inner([pl["u"], pl["v"], pl["w"]], [pl["u"], pl["v"], pl["w"]]))
    assert abs(lhs) > 1e-6 * scale
    assert abs(lhs - rhs) < 1e-12 * scale
    # the forward operator is not self-adjoint here: dropping the transpose fails
    wrong = vel_inner([-a for a in sim.advect(m, pl)], [pu["u"], pu["v"], pu["w"]])
    assert abs(lhs - wrong) > 1e-6 * scale


def test_gram_schmidt_orthonormal():
    sim = make(3)
    v, eta, _, _ = inputs.random_state(0, BOX[2], BOX[3], 8, 17, 8, 3, 0.2, 8, spectrum="k2")
    q, qe = opt.orthonormalize(sim, v, eta)
    G = np.array([[opt.inner(sim, (q[i], qe[i]), (q[j], qe[j])) for j in range(3)] for i in range(3)])
    np.testing.assert_allclose(G, 2.0 * np.eye(3), atol=1e-12)
    np.testing.assert_allclose(opt.energy(sim, q, qe), 1.0, rtol=1e-12)
    # the first member keeps its direction
    assert rel(q[0, 1:] / q[0, 1:].flat[np.argmax(np.abs(q[0, 1:]))],
               v[0, 1:] / v[0, 1:].flat[np.argmax(np.abs(q[0, 1:]))]) < 1e-12


def test_iteration_reaches_propagator_optimum():
    """One (n_x, n_z) = (1, 1) mode on laminar Couette flow, target time 5."""
    nsteps = 50
    L, NZ, N = 4, 7, 15
    dim = 2 * N
    sim = make(dim)
    v = np.zeros((dim, L, NZ, N), complex)
    eta = np.zeros_like(v)
    for j in range(N):
        v[j, 1, 1, j] = 1.0
        eta[N + j, 1, 1, j] = 1.0
    sim.v, sim.eta = v.copy(), eta.copy()
    sim.step(nsteps)
    Phi = np.concatenate([sim.v[:, 1, 1, :], sim.eta[:, 1, 1, :]], axis=1).T     # (2N, 2N)
    # energy Gram matrix of the basis (complex inner product of the mode)
    Wm = np.zeros((dim, dim), complex)
    for a in range(dim):
        for b in range(dim):
            # W[b, a] = <e_a, e_b> (complex), so that x^H W x = <s, s> for s = sum x_a e_a
            re = opt.inner(sim, (v[a], eta[a]), (v[b], eta[b]))
            im = opt.inner(sim, (1j * v[a], 1j * eta[a]), (v[b], eta[b]))
            Wm[b, a] = re - 1j * im
    Wm = 0.5 * (Wm + Wm.conj().T)
    # sigma^2 = largest eigenvalue of W^-1 Phi^H W Phi (energy-norm singular value)
    S = np.linalg.solve(Wm, Phi.conj().T @ Wm @ Phi)
    sigma2 = float(np.max(np.linalg.eigvals(S).real))
    one = make(1)
    rng = np.random.default_rng(9)
    v0 = np.zeros((1, L, NZ, N), complex)
    e0 = np.zeros_like(v0)
    v0[0, 1, 1] = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    e0[0, 1, 1] = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    gains, _, _ = opt.optimal_iteration(one, nsteps, 12, v0, e0)
    assert sigma2 > 2.0                        # transient growth of a non-normal flow
    assert abs(gains[0] / sigma2 - 1.0) < 2e-5, (gains[0], sigma2)   # measured 2.6e-6
