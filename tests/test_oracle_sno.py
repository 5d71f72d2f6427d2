"""Pins of the learned spin-up oracle (channel form, spectral neural operator,
AdamW) against library routines, closed forms and finite differences."""

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import oracle
from oracle import diagnostics as dg
from oracle import sno
from paper_2306_12739_amd import inputs

BOX = (1.75 * np.pi, 1.2 * np.pi)


def small_sim(E=2, flow=0, Nx=16, Ny=33, Nz=16):
    return oracle.OracleDNS(flow, 400.0, BOX[0], BOX[1], Nx, Ny, Nz, E, 0.02)


def test_vandermonde_matches_numpy_chebyshev():
    My = 17
    y = oracle.nodes(My)
    T = sno.chebyshev_vandermonde(My)
    ref = npcheb.chebvander(y, My - 1)
    assert np.abs(T - ref).max() <= 1e-13
    # y^3 = (3 T_1 + T_3) / 4
    a = np.linalg.solve(T, y ** 3)
    expect = np.zeros(My)
    expect[1], expect[3] = 0.75, 0.25
    assert np.abs(a - expect).max() <= 1e-13


def test_laminar_couette_channel_form():
    sim = small_sim()
    sim.set_laminar()
    ch = sno.channels_from_state(sim, *sim.get_state())
    My = sim.My
    expect = np.zeros_like(ch)
    expect[:, 1, :] = 1.0            # u = Uw y = T_1(y), same at every point
    assert np.abs(ch - expect).max() <= 1e-13


@pytest.mark.parametrize("flow", [0, 1])
def test_channel_form_round_trip(flow):
    sim = small_sim(flow=flow)
    st = inputs.random_state(flow, BOX[0], BOX[1], 16, 33, 16, 2, 0.2, 5, spectrum="k2")
    sim.set_state(*st)
    ch = sno.channels_from_state(sim, *st)
    back = sno.state_from_channels(sim, ch)
    for a, b in zip(back, st):
        assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max())


def test_projection_gives_admissible_state():
    sim = small_sim()
    rng = np.random.default_rng(3)
    ch = rng.standard_normal((2, 3 * sim.My, sim.grid.Mx * sim.grid.Mz)) * 0.1
    v, eta, U, W = sno.state_from_channels(sim, ch)
    sim.set_state(v, eta, U, W)
    vel = sim.velocities(v, eta, U, W)
    scale = max(np.abs(vel["u"]).max(), np.abs(vel["v"]).max())
    assert dg.divergence_max(sim, vel).max() <= 1e-11 * scale
    assert U[0, 0] == -1.0 and U[0, -1] == 1.0 and W[0, 0] == 0.0 and W[0, -1] == 0.0
    for f in ("u", "v", "w"):   # fluctuations vanish at the walls
        wall = vel[f][:, [0, -1]].copy()
        wall[:, :, 0, 0] = 0.0
        assert np.abs(wall).max() <= 1e-12 * scale
    # a second pass through the channel form is the identity (a projection)
    ch2 = sno.channels_from_state(sim, v, eta, U, W)
    again = sno.state_from_channels(sim, ch2)
    for a, b in zip(again, (v, eta, U, W)):
        assert np.abs(a - b).max() <= 1e-11 * max(1.0, np.abs(b).max())


def test_dft_matrices_match_numpy_fft():
    Mx, Mz, mx, mz = 12, 10, 4, 6
    rng = np.random.default_rng(0)
    h = rng.standard_normal((3, Mz * Mx))
    D, Dinv = sno.dft_matrices(Mx, Mz, mx, mz)
    X = h @ D
    F = np.fft.rfft2(h.reshape(3, Mz, Mx)) / (Mx * Mz)      # (3, Mz, Mx/2+1), [kz][kx]
    kx, kz = sno.mode_wavenumbers(mx, mz)
    ref = F[:, kz % Mz, kx]
    M = mx * mz
    assert np.abs(X[:, :M] - ref.real).max() <= 1e-14
    assert np.abs(X[:, M:] - ref.imag).max() <= 1e-14
    # inverse: real part of the half spectrum, as numpy's irfft2 does
    Y = rng.standard_normal((3, 2 * M))
    pad = np.zeros((3, Mz, Mx // 2 + 1), dtype=complex)
    pad[:, kz % Mz, kx] = Y[:, :M] + 1j * Y[:, M:]
    g_ref = np.fft.irfft2(pad, s=(Mz, Mx)) * (Mx * Mz)
    assert np.abs(Y @ Dinv - g_ref.reshape(3, -1)).max() <= 1e-12


def test_idft_inverts_dft_on_retained_band():
    Mx, Mz, mx, mz = 16, 12, 5, 8
    kxs = np.arange(Mx // 2 + 1)
    kzs = np.fft.fftfreq(Mz, 1.0 / Mz).astype(int)
    rng = np.random.default_rng(1)
    F = np.zeros((Mz, Mx // 2 + 1), dtype=complex)
    for a in range(mx):
        for kz in range(-(mz // 2) + 1, mz // 2):
            F[kz % Mz, a] = rng.standard_normal() + 1j * rng.standard_normal()
    F[:, 0] = 0.5 * (F[:, 0] + np.conj(F[(-kzs) % Mz, 0]))
    F[0, 0] = F[0, 0].real
    h = np.fft.irfft2(F, s=(Mz, Mx)).ravel()
    D, Dinv = sno.dft_matrices(Mx, Mz, mx, mz)
    assert np.abs((h @ D) @ Dinv - h).max() <= 1e-12 * np.abs(h).max()
    del kxs


def test_gelu_values_and_derivative():
    assert abs(sno.gelu(np.array(1.0)) - 0.8413447460685429) <= 1e-15
    assert sno.gelu(np.array(0.0)) == 0.0
    assert abs(sno.gelu(np.array(8.0)) - 8.0) <= 1e-12
    z = np.linspace(-4, 4, 33)
    e = 1e-6
    fd = (sno.gelu(z + e) - sno.gelu(z - e)) / (2 * e)
    assert np.abs(fd - sno.gelu_grad(z)).max() <= 1e-9


def tiny():
    cfg = sno.SNOConfig(channels=5, width=4, layers=2, Mx=8, Mz=6, mx=3, mz=4)
    rng = np.random.default_rng(11)
    theta = rng.standard_normal(cfg.num_params()) * 0.3
    x = rng.standard_normal((3, cfg.C, cfg.P))
    y = x + 0.3 * rng.standard_normal(x.shape)
    return cfg, theta, x, y


def test_sno_gradient_matches_finite_differences():
    cfg, theta, x, y = tiny()

    def L(t):
        return sno.rel_l2_loss(sno.forward(cfg, t, x)[0], y)[0]

    yhat, cache = sno.forward(cfg, theta, x)
    _, dy = sno.rel_l2_loss(yhat, y)
    g = sno.backward(cfg, theta, cache, dy)
    e = 1e-6
    offs = 0
    for name, sh in cfg.shapes():      # a few coordinates of every parameter block
        n = int(np.prod(sh))
        for i in np.unique(np.linspace(0, n - 1, 4).astype(int)):
            d = np.zeros_like(theta)
            d[offs + i] = e
            fd = (L(theta + d) - L(theta - d)) / (2 * e)
            assert abs(fd - g[offs + i]) <= 1e-7 + 1e-5 * abs(fd), (name, i, fd, g[offs + i])
        offs += n
    # and along a random direction through all parameters
    u = np.random.default_rng(2).standard_normal(theta.shape)
    fd = (L(theta + e * u) - L(theta - e * u)) / (2 * e)
    assert abs(fd - g @ u) <= 1e-6 * max(1.0, abs(fd))


def test_loss_properties():
    rng = np.random.default_rng(4)
    y = rng.standard_normal((2, 3, 5))
    assert sno.rel_l2_loss(y, y)[0] == 0.0
    yh = y + rng.standard_normal(y.shape)
    a = sno.rel_l2_loss(yh, y)[0]
    b = sno.rel_l2_loss(7.0 * yh, 7.0 * y)[0]
    assert abs(a - b) <= 1e-14
    one = sno.rel_l2_loss(yh[:1], y[:1])[0]
    assert abs(one - np.linalg.norm(yh[0] - y[0]) / np.linalg.norm(y[0])) <= 1e-14


def test_adamw_first_step_closed_form():
    rng = np.random.default_rng(5)
    w = rng.standard_normal(10)
    g = rng.standard_normal(10)
    lr, wd, eps = 1e-3, 1e-2, 1e-8
    w1, m, v = sno.adamw_step(w, g, np.zeros(10), np.zeros(10), 1, lr, weight_decay=wd, eps=eps)
    assert np.abs(w1 - (w - lr * wd * w - lr * g / (np.abs(g) + eps))).max() <= 1e-15
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # zero gradient: only the decoupled decay acts
    w2, _, _ = sno.adamw_step(w, np.zeros(10), np.zeros(10), np.zeros(10), 1, lr, weight_decay=wd)
    assert np.abs(w2 - w * (1 - lr * wd)).max() <= 1e-15
