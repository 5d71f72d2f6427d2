"""Pins of the Helmholtz-Poisson (KMM) v discretization (CPU).

Both v discretizations (the paper's clamped fourth-derivative operator and
the Helmholtz-Poisson system for phi = Lap v with clamped walls) must reproduce
the Stokes eigenvalues of the clamped plane channel, which are closed-form
roots of transcendental equations: v = cos(p y)/cos p - cosh(k y)/cosh k
(even, p tan p = -k tanh k) and v = sin(p y)/sin p - sinh(k y)/sinh k (odd,
p cot p = k coth k), with Lap Lap v = mu Lap v, mu = -(k^2 + p^2).  The CN factor
a of an eigenvector gives mu = (a - 1) / (c (a + 1)).  The two discretizations
differ by a collocation error that falls faster than any power of 1/Ny
(checked on the steady forced problem).
"""

import numpy as np
from scipy.optimize import brentq

import oracle
from oracle.cheb import diff_matrix, nodes
from oracle.operators import kmm_v_operators


def stokes_mu(k, parity, branch=0):
    if parity == "even":
        f = lambda p: p * np.tan(p) + k * np.tanh(k)
        lo, hi = np.pi / 2 + branch * np.pi, np.pi + branch * np.pi
    else:
        f = lambda p: p / np.tan(p) - k / np.tanh(k)
        lo, hi = np.pi + branch * np.pi, 1.5 * np.pi + branch * np.pi
    p = brentq(f, lo + 1e-12, hi - 1e-12)
    return -(k * k + p * p)


def discrete_mus(A, c):
    a = np.linalg.eigvals(A)
    return np.sort(((a - 1) / (c * (a + 1))).real)[::-1]


def test_stokes_eigenvalues_both_discretizations():
    k2, dt, Re = 1.7, 0.02, 500.0
    c = dt / (2 * Re)
    k = np.sqrt(k2)
    exact = sorted([stokes_mu(k, "even", 0), stokes_mu(k, "odd", 0), stokes_mu(k, "even", 1)], reverse=True)
    My = 25
    y = nodes(My)
    D1 = diff_matrix(y)
    A_kmm, _ = kmm_v_operators(D1, D1 @ D1, k2, c)
    sim = oracle.OracleDNS(0, Re, 2 * np.pi / k, 2 * np.pi, 4, My, 4, 1, dt)
    A_cl = sim.ops.modes[1.0][(1, 0)].A_v
    for A in (A_kmm, A_cl):
        mus = discrete_mus(A, c)[:3]
        np.testing.assert_allclose(mus, exact, rtol=1e-9)


def test_kmm_converges_to_clamped_spectrally():
    """Steady forced Stokes problem, Lap Lap v = -Re f with clamped walls: the
    CN fixed points v* = (I - A_v)^-1 (h dt B_v f) of both discretizations
    converge to each other faster than any power of 1/Ny for an analytic f.
    (Trajectories at a fixed dt converge only algebraically: CN does not damp
    the stiffest discrete modes, whose share of the initial data the two
    discretizations resolve differently.)"""
    k2, dt, Re = 1.7, 0.02, 500.0
    c = dt / (2 * Re)
    gaps = []
    for My in (9, 13, 17):
        y = nodes(My)
        D1 = diff_matrix(y)
        A_k, B_k = kmm_v_operators(D1, D1 @ D1, k2, c)
        sim = oracle.OracleDNS(0, Re, 2 * np.pi / np.sqrt(k2), 2 * np.pi, 4, My, 4, 1, dt)
        op = sim.ops.modes[1.0][(1, 0)]
        yi = y[1:-1]
        f = np.cos(yi) + 0.3 * np.exp(yi)
        I = np.eye(My - 2)
        vk = np.linalg.solve(I - A_k, B_k @ f)
        vc = np.linalg.solve(I - op.A_v, op.B_v @ f)
        gaps.append(np.linalg.norm(vk - vc) / np.linalg.norm(vc))
    assert gaps[0] > 1e-7
    assert gaps[1] < 1e-3 * gaps[0] and gaps[2] < 1e-10, gaps


def test_kmm_nonlinear_run_close_to_clamped():
    from paper_2306_12739_amd import inputs
    st = inputs.workload_state("couette-re400-16x33x16-e2")
    out = []
    for vd in ("clamped", "kmm"):
        sim = oracle.OracleDNS(0, 400.0, 1.75 * np.pi, 1.2 * np.pi, 16, 33, 16, 2, 0.02, v_discretization=vd)
        sim.set_state(*st)
        sim.step(10)
        out.append(sim.v)
    d = np.linalg.norm(out[1] - out[0]) / np.linalg.norm(out[0])
    assert 0 < d < 1e-6
