"""Planted mistakes in the oracle must be caught by the pins (CPU only).

Each test patches one plausible slip into a copy of the oracle's arithmetic (a
dropped term, a flipped sign, a transposed operand) and checks that one of the
physics pins of test_oracle_physics.py or of the statistics pins of
test_oracle_statistics.py then fails.
"""

import numpy as np
import pytest

import oracle
from oracle import diagnostics as dg
from oracle.step import OracleDNS
import test_oracle_physics as phys
import test_oracle_statistics as stats_pins


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


# ---- one-point statistics and power input (pins in test_oracle_statistics.py) ----


def _result_with(fluct_about_member_mean=False, drop_mean_term=False, tau_sign=1.0, mean_of_rms=False):
    """A copy of StatsAccumulator.result with one planted slip."""
    def result(self, sim):
        m = {k: v / self.n for k, v in self.sums.items()}
        if fluct_about_member_mean or mean_of_rms:
            U, W, U2, W2 = m["U"], m["W"], m["U2"], m["W2"]       # per member
        else:
            U, W = m["U"].mean(axis=0), m["W"].mean(axis=0)
            U2, W2 = m["U2"].mean(axis=0), m["W2"].mean(axis=0)
        uu, vv, ww, uv = m["uu"], m["vv"], m["ww"], m["uv"]
        if not (fluct_about_member_mean or mean_of_rms):
            uu, vv, ww, uv = (a.mean(axis=0) for a in (uu, vv, ww, uv))
        extra_u = 0.0 if drop_mean_term else U2 - U ** 2
        extra_w = 0.0 if drop_mean_term else W2 - W ** 2
        out = {
            "U": U, "W": W,
            "urms": np.sqrt(np.maximum(uu + extra_u, 0.0)),
            "vrms": np.sqrt(np.maximum(vv, 0.0)),
            "wrms": np.sqrt(np.maximum(ww + extra_w, 0.0)),
            "uv": uv,
        }
        if fluct_about_member_mean or mean_of_rms:
            out = {k: v.mean(axis=0) for k, v in out.items()}
        lo, hi = m["dUlo"].mean(), m["dUhi"].mean()
        tau = 0.5 * (abs(lo) + abs(hi)) / sim.Re if sim.flow == 0 else tau_sign * (lo - hi) / (2.0 * sim.Re)
        out["tau_w"] = tau
        out["Re_tau"] = sim.Re * np.sqrt(abs(tau))
        return out
    return result


def test_dropped_mean_profile_fluctuation_is_caught(monkeypatch):
    monkeypatch.setattr(dg.StatsAccumulator, "result", _result_with(drop_mean_term=True))
    stats_pins.check_laminar_couette()          # unaffected: no mean fluctuations
    with pytest.raises(AssertionError):
        stats_pins.check_mean_offsets_are_fluctuations()


def test_fluctuations_about_each_members_mean_are_caught(monkeypatch):
    monkeypatch.setattr(dg.StatsAccumulator, "result", _result_with(fluct_about_member_mean=True))
    with pytest.raises(AssertionError):
        stats_pins.check_mean_offsets_are_fluctuations()


def test_mean_of_member_rms_is_caught(monkeypatch):
    monkeypatch.setattr(dg.StatsAccumulator, "result", _result_with(mean_of_rms=True))
    with pytest.raises(AssertionError):
        stats_pins.check_rms_pools_members()


def test_channel_wall_shear_sign_is_caught(monkeypatch):
    monkeypatch.setattr(dg.StatsAccumulator, "result", _result_with(tau_sign=-1.0))
    stats_pins.check_laminar_couette()          # Couette branch untouched
    with pytest.raises(AssertionError):
        stats_pins.check_laminar_channel()


def test_unweighted_parseval_sum_is_caught(monkeypatch):
    def profiles(sim, vel=None):
        vel = sim.velocities(sim.v, sim.eta, sim.U, sim.W) if vel is None else vel
        mask = np.ones_like(sim.grid.mk)           # slip: n_x >= 1 modes counted once
        mask[0, 0] = 0.0

        def s(a, b=None):
            b = a if b is None else b
            return np.einsum("lm,ejlm->ej", mask, np.real(a * np.conj(b)))
        return {"U": sim.U.copy(), "W": sim.W.copy(), "uu": s(vel["u"]), "vv": s(vel["v"]),
                "ww": s(vel["w"]), "uv": s(vel["u"], vel["v"])}
    monkeypatch.setattr(dg, "profiles", profiles)
    with pytest.raises(AssertionError):
        stats_pins.check_profiles_match_physical_average()


def test_channel_power_without_height_is_caught(monkeypatch):
    orig = dg.power_input

    def bad(sim):
        p = orig(sim)
        return p * dg.LY if sim.flow == 1 else p    # slip: gamma Q instead of gamma Q / Ly
    monkeypatch.setattr(dg, "power_input", bad)
    with pytest.raises(AssertionError):
        stats_pins.check_channel_budget()
    with pytest.raises(AssertionError):
        stats_pins.check_laminar_power_balance()


def test_channel_power_sign_is_caught(monkeypatch):
    orig = dg.power_input

    def bad(sim):
        p = orig(sim)
        return -p if sim.flow == 1 else p
    monkeypatch.setattr(dg, "power_input", bad)
    with pytest.raises(AssertionError):
        stats_pins.check_channel_budget()
