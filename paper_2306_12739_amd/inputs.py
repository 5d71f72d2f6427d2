"""Seeded synthetic initial conditions for ensemble runs.

This module is shared by the tests, the benchmark and the oracle checks.  It
holds none of the solver's arithmetic: it only evaluates smooth random
functions that satisfy the wall conditions of the problem statement (Sec. 2,
Eq. (b_ve): v = dv/dy = eta = 0 at both walls) on the Chebyshev-Gauss-Lobatto
grid, and returns them in the library's host state layout

  v, eta : complex (E, Nx/2, Nz-1, Ny-2)   [member][kx][kz in FFT order][interior j]
  U, W   : real    (E, Ny)                 [member][j], walls included.

Recipe (the paper initialises its ensembles from perturbed copies of a
turbulent state, Sec. 4.2; these synthetic fields stand in for that):
  v_k(y)   = A s_k sum_n a_{k,n} sig_n (1 - y^2)^2 T_n(y)
  eta_k(y) = A s_k |k| sum_n b_{k,n} sig_n (1 - y^2) T_n(y)
with complex Gaussian a, b.  ``spectrum="low"`` excites 0 <= n_x < nlow,
|n_z| < nlow (not the mean) with s_k = 1 and Chebyshev degrees n < 4;
``spectrum="k2"`` excites every kept mode with s_k = 1/max(|k|, k_min)
(energy ~ k^-2) and all degrees with sig_n = (n + 1)^-2.  The n_x = 0 column is
made Hermitian.  The amplitude A is the rms over interior nodes and the
Parseval-weighted half spectrum of (v, eta / |k|), both velocity-sized, scaled
to ``amplitude`` times the laminar reference speed (1).  U is the laminar
profile (Couette U = Uw y, channel U = 1 - y^2) and W = 0.
"""

import numpy as np


def gauss_lobatto(Ny):
    j = np.arange(Ny)
    return -np.cos(np.pi * j / (Ny - 1))


def _cheb_T(n, y):
    return np.cos(n * np.arccos(np.clip(y, -1.0, 1.0)))


def laminar_profile(flow, Ny, Uw=1.0):
    y = gauss_lobatto(Ny)
    return Uw * y if flow == 0 else 1.0 - y ** 2


def random_state(flow, Lx, Lz, Nx, Ny, Nz, ensemble, amplitude, seed,
                 spectrum="low", nlow=4, Uw=1.0):
    rng = np.random.default_rng(seed)
    y = gauss_lobatto(Ny)
    yi = y[1:-1]
    N = Ny - 2
    L = Nx // 2
    P = Nz // 2
    NZ = Nz - 1
    iz = np.arange(NZ)
    nz = np.where(iz < P, iz, iz - NZ)
    nx = np.arange(L)
    kx = 2.0 * np.pi * nx / Lx
    kz = 2.0 * np.pi * nz / Lz
    kk = np.sqrt(kx[:, None] ** 2 + kz[None, :] ** 2)           # (L, NZ)
    if spectrum == "low":
        mask = (nx[:, None] < nlow) & (np.abs(nz)[None, :] < nlow)
        degs = np.arange(min(4, N))
        sig = np.ones(len(degs))
        shape = np.ones((L, NZ))
    elif spectrum == "k2":
        mask = np.ones((L, NZ), dtype=bool)
        degs = np.arange(N)
        sig = (degs + 1.0) ** -2
        kmin = 2.0 * np.pi / max(Lx, Lz)
        shape = 1.0 / np.maximum(kk, kmin)
    else:
        raise ValueError(spectrum)
    mask[0, 0] = False
    T = np.stack([_cheb_T(n, yi) for n in degs])               # (nd, N)
    bv = (1.0 - yi ** 2) ** 2 * T                               # (nd, N)
    be = (1.0 - yi ** 2) * T
    E = ensemble
    shp = (E, L, NZ, len(degs))
    a = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * sig
    b = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * sig
    v = np.einsum("elmn,nj->elmj", a, bv) * (shape * mask)[None, :, :, None]
    eta = np.einsum("elmn,nj->elmj", b, be) * (shape * kk * mask)[None, :, :, None]
    # Hermitian n_x = 0 column: the (0, -n_z) entry mirrors (0, n_z).
    for i in range(1, P):
        v[:, 0, NZ - i] = np.conj(v[:, 0, i])
        eta[:, 0, NZ - i] = np.conj(eta[:, 0, i])
    # amplitude: rms of (v, eta/|k|) over interior nodes and the half spectrum
    mk = np.where(nx[:, None] == 0, 1.0, 2.0) * np.ones(NZ)[None, :]
    ksafe = np.where(kk > 0, kk, 1.0)
    for e in range(E):
        q = (mk[:, :, None] * (np.abs(v[e]) ** 2 + np.abs(eta[e] / ksafe[:, :, None]) ** 2)).sum(axis=(0, 1))
        rms = np.sqrt(q.mean())
        if rms > 0:
            v[e] *= amplitude / rms
            eta[e] *= amplitude / rms
    U = np.tile(laminar_profile(flow, Ny, Uw), (E, 1))
    W = np.zeros((E, Ny))
    return v, eta, U, W


# Named workloads (box, grid, ensemble, time step, initial condition).
# Channel Reynolds number 4200 is the laminar-centreline value whose bulk
# Reynolds number (2h U_b / nu with U_b = 2/3) is 5600.
WORKLOADS = {
    "couette-re400-16x33x16-e2": dict(
        flow=0, Re=400.0, Lx=1.75 * np.pi, Lz=1.2 * np.pi, Nx=16, Ny=33, Nz=16,
        ensemble=2, dt=0.02, steps=100, amplitude=0.1, spectrum="low", seed=1000),
    "couette-re600-32x49x32-e64": dict(
        flow=0, Re=600.0, Lx=1.75 * np.pi, Lz=1.2 * np.pi, Nx=32, Ny=49, Nz=32,
        ensemble=64, dt=0.02, steps=2000, amplitude=0.2, spectrum="k2", seed=1001),
    "channel-re4200-64x97x64-e16": dict(
        flow=1, Re=4200.0, Lx=2.0 * np.pi, Lz=np.pi, Nx=64, Ny=97, Nz=64,
        ensemble=16, dt=0.005, steps=1000, amplitude=0.3, spectrum="k2", seed=1002),
    # paper-resolution grids (72 x 73 x 72 on the 108 x 73 x 108 grid), box 2 pi x 2 x pi, dt = 0.008
    "channel-re4200-72x73x72-e16": dict(
        flow=1, Re=4200.0, Lx=2.0 * np.pi, Lz=np.pi, Nx=72, Ny=73, Nz=72,
        ensemble=16, dt=0.008, steps=50000, amplitude=0.3, spectrum="k2", seed=1008),
    "couette-re3000-72x73x72-e16": dict(
        flow=0, Re=3000.0, Lx=2.0 * np.pi, Lz=np.pi, Nx=72, Ny=73, Nz=72,
        ensemble=16, dt=0.008, steps=50000, amplitude=0.3, spectrum="k2", seed=1009),
}


# Uneven batched ensemble: three Couette groups of different Re and grid in one
# step call (members 64 / 40 / 24, 500 steps each); per-group seeds 1003 + g.
GROUPED_WORKLOADS = {
    "couette-grouped-re400-600-1000-e128": dict(
        steps=500,
        groups=[
            dict(flow=0, Re=400.0, Lx=1.75 * np.pi, Lz=1.2 * np.pi, Nx=16, Ny=33, Nz=16,
                 members=64, dt=0.02, amplitude=0.2, spectrum="k2", seed=1003),
            dict(flow=0, Re=600.0, Lx=1.75 * np.pi, Lz=1.2 * np.pi, Nx=32, Ny=49, Nz=32,
                 members=40, dt=0.02, amplitude=0.2, spectrum="k2", seed=1004),
            dict(flow=0, Re=1000.0, Lx=1.75 * np.pi, Lz=1.2 * np.pi, Nx=48, Ny=65, Nz=48,
                 members=24, dt=0.02, amplitude=0.2, spectrum="k2", seed=1005),
        ]),
}


def group_state(group, members=None, seed=None):
    """Initial state of one group of a grouped workload."""
    g = group
    return random_state(g["flow"], g["Lx"], g["Lz"], g["Nx"], g["Ny"], g["Nz"],
                        g["members"] if members is None else members, g["amplitude"],
                        g["seed"] if seed is None else seed, spectrum=g["spectrum"])


def workload_state(name, ensemble=None, seed=None):
    w = WORKLOADS[name]
    return random_state(w["flow"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"],
                        w["ensemble"] if ensemble is None else ensemble,
                        w["amplitude"], w["seed"] if seed is None else seed,
                        spectrum=w["spectrum"])
