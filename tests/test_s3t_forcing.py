"""Host logic of the S3T driver (CPU; the library's host operator builder only).

The forcing structures must be eigenvectors of the viscous operators the step
uses, scaled to equal dissipation rates, and realizations must touch only the
forced streamwise wavenumber; the growth-rate fit must recover a known rate.
"""

import numpy as np

from paper_2306_12739_amd import s3t

SMALL = dict(flow=0, Re=1000.0, Lx=2.0 * np.pi, Lz=1.2 * np.pi, Nx=16, Ny=25, Nz=16,
             ensemble=3, dt=0.02, forced_nx=1, energy_ratio=1e-3, seed=1)


def test_structures_are_scaled_diffusion_eigenvectors():
    f = s3t.Forcing(SMALL, 1)
    w = SMALL
    c = w["dt"] / (2 * w["Re"])
    N = w["Ny"] - 2
    import paper_2306_12739_amd.dns as dns
    ops = dns.host_operators(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], w["dt"], 1)
    P = w["Nz"] // 2
    for iz, bv, be in f.modes[:5]:
        nz = iz if iz < P else iz - (w["Nz"] - 1)
        kx, kz = 2 * np.pi / w["Lx"], 2 * np.pi * nz / w["Lz"]
        k2 = kx * kx + kz * kz
        g = P + abs(nz)
        Av, Ae = ops["ops"][g, 0], ops["ops"][g, 2]
        # Lap_D from the eta operator, L from the v operator (CN: A = (I + cX)(I - cX)^-1)
        Lap = np.linalg.solve(Ae + np.eye(N), Ae - np.eye(N)) / c
        Lv = np.linalg.solve(Av + np.eye(N), Av - np.eye(N)) / c
        assert bv.shape == (N, N) and be.shape == (N, N)
        rates_v, rates_e = [], []
        for fv in bv:
            phi = np.linalg.solve(Lap, fv)                 # the structure as v
            mu = (phi @ (Lv @ phi)) / (phi @ phi)
            assert np.linalg.norm(Lv @ phi - mu * phi) <= 1e-6 * abs(mu) * np.linalg.norm(phi)
            rates_v.append(2 * abs(mu) * f.energy_v(phi, k2) / w["Re"])
        for fe in be:
            lam = (fe @ (Lap @ fe)) / (fe @ fe)
            assert np.linalg.norm(Lap @ fe - lam * fe) <= 1e-8 * abs(lam) * np.linalg.norm(fe)
            rates_e.append(2 * abs(lam) * f.energy_eta(fe, k2) / w["Re"])
        np.testing.assert_allclose(rates_v, 1.0, rtol=1e-6)
        np.testing.assert_allclose(rates_e, 1.0, rtol=1e-8)


def test_realizations_force_one_streamwise_wavenumber():
    f = s3t.Forcing(SMALL, 1)
    rng = np.random.default_rng(3)
    fv, fe = f.realization(rng, 3, 2.0)
    assert fv.shape == (3, 8, 15, 23) and fe.shape == fv.shape
    mask = np.ones(8, bool)
    mask[1] = False
    assert np.abs(fv[:, mask]).max() == 0.0 and np.abs(fe[:, mask]).max() == 0.0
    assert np.abs(fv[:, 1]).min() >= 0.0 and np.abs(fv[:, 1]).max() > 0.0
    # members draw independent realizations
    assert np.linalg.norm(fv[0] - fv[1]) > 0.1 * np.linalg.norm(fv[0])


def test_mode_energy_of_a_single_streak():
    w = SMALL
    f = s3t.Forcing(w, 1)
    N = w["Ny"] - 2
    y = -np.cos(np.pi * np.arange(1, w["Ny"] - 1) / (w["Ny"] - 1))
    v = np.zeros((1, 8, 15, N), complex)
    eta = np.zeros_like(v)
    eta[0, 0, 1] = (1 - y ** 2)
    eta[0, 0, 14] = (1 - y ** 2)
    pert, rs = s3t.mode_energy(w, f.D1c, f.ccw, v, eta)
    kz = 2 * np.pi / w["Lz"]
    # two modes (+-kz), each (1/4) int (1 - y^2)^2 / kz^2 dy = (1/4)(16/15) / kz^2
    np.testing.assert_allclose(rs[0], 2 * 0.25 * (16 / 15) / kz ** 2, rtol=1e-12)
    assert pert[0] == 0.0


def test_growth_rate_fit():
    t = np.linspace(0, 400, 200)
    e = np.minimum(1e-14 * np.exp(2 * 0.03 * t), 2e-2) * (1 + 0.01 * np.sin(t))
    assert abs(s3t.growth_rate(t, e) - 0.03) < 2e-3
    assert s3t.growth_rate(t, np.full_like(t, 1e-3)) is None
