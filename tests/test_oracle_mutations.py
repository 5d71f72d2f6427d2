"""Planted mistakes in the oracle must be caught by the pins (CPU only).

Each test patches one plausible slip into a copy of the oracle's arithmetic (a
dropped term, a flipped sign, a transposed operand) and checks that one of the
physics pins of test_oracle_physics.py then fails.
"""

import numpy as np
import pytest

import oracle
from oracle import diagnostics as dg
from oracle.step import OracleDNS
import test_oracle_physics as phys


def budget_residual(sim, nsteps=8):
    dt = sim.dt
    E0 = dg.energy(sim)
    b0 = dg.power_input(sim) - dg.dissipation(sim)
    worst = 0.0
    for _ in range(nsteps):
        sim.step(1)
        E1 = dg.energy(sim)
        b1 = dg.power_input(sim) - dg.dissipation(sim)
        worst = max(worst, float(np.max(np.abs(((E1 - E0) / dt - 0.5 * (b0 + b1)) / dg.dissipation(sim)))))
        E0, b0 = E1, b1
    return worst


def run_budget():
    sim = phys.cfg1_sim(E=1)
    sim.set_state(*phys.inputs.workload_state("couette-re400-16x33x16-e2", ensemble=1))
    return budget_residual(sim)


def test_unmutated_budget_passes():
    assert run_budget() <= 1e-3


def test_sign_flip_in_eta_forcing_is_caught(monkeypatch):
    orig = OracleDNS.rhs

    def bad(self, *a):
        F, G, EU, EW = orig(self, *a)
        return F, -G, EU, EW
    monkeypatch.setattr(OracleDNS, "rhs", bad)
    assert run_budget() > 1e-3


def test_transposed_y_derivative_in_mean_forcing_is_caught(monkeypatch):
    orig = OracleDNS.rhs

    def bad(self, Nu, Nv, Nw, uv, wv):
        F, G, _, _ = orig(self, Nu, Nv, Nw, uv, wv)
        D1 = self.ops.D1
        return F, G, -(uv @ D1)[:, 1:-1], -(wv @ D1)[:, 1:-1]
    monkeypatch.setattr(OracleDNS, "rhs", bad)
    assert run_budget() > 1e-3


def test_dropped_horizontal_laplacian_term_is_caught(monkeypatch):
    orig = OracleDNS.rhs

    def bad(self, Nu, Nv, Nw, uv, wv):
        F, G, EU, EW = orig(self, Nu, Nv, Nw, uv, wv)
        g = self.grid
        F = F + np.moveaxis((g.K2 * Nv)[:, 1:-1], 1, -1)     # undo the -k^2 N_v term
        return F, G, EU, EW
    monkeypatch.setattr(OracleDNS, "rhs", bad)
    with pytest.raises(AssertionError):
        phys.test_tollmien_schlichting_growth_rate()


def test_wrong_cn_fraction_is_caught(monkeypatch):
    orig = OracleDNS.solve

    def bad(self, h, x0, Xc):
        return orig(self, 1.0 if h == 0.5 else h, x0, Xc)
    monkeypatch.setattr(OracleDNS, "solve", bad)
    with pytest.raises(AssertionError):
        phys.test_tollmien_schlichting_growth_rate()
