"""GPU parity of the rotational advection form (omega x u) against the oracle's
rotational form, through the C ABI.

Bars as for the advective form: stage intermediates 1e-12 (FP64) / 2e-6 (FP32
FFT arithmetic) relative per field, states 1e-10 relative after 100 FP64
steps; the mixed path within 1e-4 of the FP64 oracle after 100 steps.  Every
plane-kernel chunk-row variant of every grid is checked; the 64x97x64 channel
is stepped at its full ensemble size and compared on sampled members.
"""

import sys

import numpy as np
import pytest

import oracle
from oracle import diagnostics as dg
from paper_2306_12739_amd import dns, inputs

pytestmark = pytest.mark.gpu

GRIDS = [  # (flow, Re, Lx, Lz, N, Ny, dt, amplitude)
    (0, 400.0, 1.75 * np.pi, 1.2 * np.pi, 16, 33, 0.02, 0.1),
    (0, 600.0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 0.02, 0.2),
    (0, 1000.0, 1.75 * np.pi, 1.2 * np.pi, 48, 65, 0.02, 0.2),
    (1, 4200.0, 2.0 * np.pi, np.pi, 64, 97, 0.005, 0.3),
]
ROWS = {
    dns.PREC_FP64: {16: [24, 12, 8], 32: [16, 24, 8], 48: [12, 8], 64: [16, 12, 8]},
    dns.PREC_MIXED_FP32: {16: [24, 12, 8], 32: [16, 24, 48], 48: [12, 24, 36], 64: [32, 24, 16]},
}
CFG1 = inputs.WORKLOADS["couette-re400-16x33x16-e2"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def pair(flow, Re, Lx, Lz, n, Ny, E, dt, st):
    gpu = dns.Ensemble(flow, Re, Lx, Lz, n, Ny, n, E, dt)
    gpu.set_advection(dns.ADV_ROTATIONAL)
    gpu.set_state(*st)
    ref = oracle.OracleDNS(flow, Re, Lx, Lz, n, Ny, n, E, dt, advection="rotational")
    ref.set_state(*st)
    return gpu, ref


@pytest.mark.parametrize("precision", [dns.PREC_FP64, dns.PREC_MIXED_FP32])
@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: f"{g[4]}x{g[5]}")
def test_rotational_terms_every_variant(grid, precision):
    flow, Re, Lx, Lz, n, Ny, dt, amp = grid
    st = inputs.random_state(flow, Lx, Lz, n, Ny, n, 2, amp, 2025, spectrum="k2")
    gpu, ref = pair(flow, Re, Lx, Lz, n, Ny, 2, dt, st)
    gpu.set_precision(precision)
    rv = ref.velocities(ref.v, ref.eta, ref.U, ref.W)
    Nu, Nv, Nw, uv, wv = ref.nonlinear_rotational(rv)
    tol = 1e-12 if precision == dns.PREC_FP64 else 2e-6
    for rows in ROWS[precision][n]:
        say(f"case: rotational plane variant rows={rows}, grid {n}x{Ny}x{n}, precision {precision}")
        gpu.set_option(dns.OPT_PLANE_ROWS, rows)
        _, nl, means = gpu.debug_stage0()
        errs = [rel(nl[i], f) for i, f in enumerate((Nu, Nv, Nw))]
        say("  errors", errs)
        assert max(errs) <= tol, (rows, errs)
        mtol = (1e-13 if precision == dns.PREC_FP64 else 1e-6) * max(1.0, np.abs(uv).max())
        assert np.abs(means[0] - uv).max() <= mtol
        assert np.abs(means[1] - wv).max() <= mtol
    gpu.close()


def test_rotational_parity_couette_100_steps_fp64():
    say("case: rotational form, couette 16x33x16 E=2 FP64, 100 steps dt=0.02")
    w = CFG1
    st = inputs.workload_state("couette-re400-16x33x16-e2")
    gpu, ref = pair(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], 2, w["dt"], st)
    gpu.step(100)
    ref.step(100)
    v, eta, U, W = gpu.get_state()
    lam = ref.laminar_profile()[None, :]
    errs = {"v": rel(v, ref.v), "eta": rel(eta, ref.eta), "U-Ulam": rel(U - lam, ref.U - lam),
            "W": rel(W, ref.W) if np.any(ref.W) else np.abs(W).max()}
    say("errors after 100 steps:", errs)
    for k, e in errs.items():
        assert e <= 1e-10, (k, e)
    s = gpu.stats()
    np.testing.assert_allclose(s["energy"], dg.energy(ref), rtol=1e-12)
    np.testing.assert_allclose(s["dissipation"], dg.dissipation_vorticity(ref), rtol=1e-11)
    gpu.close()


def test_rotational_parity_channel_fp64_ragged_members():
    say("case: rotational form, channel 32x49x32 Re=2000 E=5 FP64, 10 steps dt=0.01")
    st = inputs.random_state(1, 2 * np.pi, np.pi, 32, 49, 32, 5, 0.3, 41, spectrum="k2")
    gpu, ref = pair(1, 2000.0, 2 * np.pi, np.pi, 32, 49, 5, 0.01, st)
    gpu.step(10)
    ref.step(10)
    v, eta, U, W = gpu.get_state()
    lam = ref.laminar_profile()[None, :]
    errs = {"v": rel(v, ref.v), "eta": rel(eta, ref.eta), "U-Ulam": rel(U - lam, ref.U - lam),
            "W": rel(W, ref.W)}
    say("errors:", errs)
    for k, e in errs.items():
        assert e <= 1e-10, (k, e)
    np.testing.assert_allclose(gpu.stats()["flux"], 4.0 / 3.0, rtol=1e-13)
    gpu.close()


def test_rotational_channel_64x97x64_sampled_members_mixed():
    """Full bench size in the benchmark's launch configuration (mixed, graph,
    member chains); members 0 and 15 against the FP64 oracle after 2 steps."""
    say("case: rotational form, channel 64x97x64 E=16 mixed graph, 2 steps, members 0 and 15")
    name = "channel-re4200-64x97x64-e16"
    w = inputs.WORKLOADS[name]
    st = inputs.workload_state(name)
    gpu = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], 16, w["dt"])
    gpu.set_advection(dns.ADV_ROTATIONAL)
    gpu.set_precision(dns.PREC_MIXED_FP32)
    gpu.set_option(dns.OPT_GRAPH, 1)
    gpu.set_state(*st)
    pick = [0, 15]
    ref = oracle.OracleDNS(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], 2, w["dt"],
                           advection="rotational")
    ref.set_state(*(a[pick] for a in st))
    gpu.step(2)
    ref.step(2)
    v, eta, U, W = gpu.get_state()
    lam = ref.laminar_profile()[None, :]
    errs = {"v": rel(v[pick], ref.v), "eta": rel(eta[pick], ref.eta),
            "U-Ulam": rel(U[pick] - lam, ref.U - lam), "W": rel(W[pick], ref.W)}
    say("errors:", errs)
    for k, e in errs.items():
        assert e <= 1e-5, (k, e)
    s = gpu.stats()
    assert not s["failed"].any()
    np.testing.assert_allclose(s["flux"], 4.0 / 3.0, rtol=1e-12)
    gpu.close()


def test_rotational_mixed_100_steps():
    say("case: rotational form mixed FP32, couette 16x33x16, 100 steps vs FP64 oracle")
    w = CFG1
    st = inputs.workload_state("couette-re400-16x33x16-e2")
    gpu, ref = pair(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], 2, w["dt"], st)
    gpu.set_precision(dns.PREC_MIXED_FP32)
    gpu.step(100)
    ref.step(100)
    v, eta, U, W = gpu.get_state()
    lam = ref.laminar_profile()[None, :]
    errs = {"v": rel(v, ref.v), "eta": rel(eta, ref.eta), "U-Ulam": rel(U - lam, ref.U - lam)}
    say("errors after 100 steps:", errs)
    assert max(errs.values()) <= 1e-4
    gpu.close()


def test_form_switch_between_steps_and_graph():
    """Switching the form between steps re-captures the graph; the run equals
    one that used each form eagerly for the same steps (bitwise)."""
    say("case: advective 2 steps then rotational 2 steps, graph vs eager, couette 32x49x32 E=3")
    st = inputs.random_state(0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, 3, 0.2, 43, spectrum="k2")
    out = []
    for graph in (1, 0):
        ens = dns.Ensemble(0, 600.0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, 3, 0.02)
        ens.set_option(dns.OPT_GRAPH, graph)
        ens.set_state(*st)
        ens.step(2)
        ens.set_advection(dns.ADV_ROTATIONAL)
        ens.step(2)
        out.append(ens.get_state())
        with pytest.raises(dns.DnsError):
            ens.set_advection(2)
        ens.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)
    ref = oracle.OracleDNS(0, 600.0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, 3, 0.02)
    ref.set_state(*st)
    ref.step(2)
    ref.advection = "rotational"
    ref.step(2)
    assert rel(out[0][0], ref.v) <= 1e-10 and rel(out[0][1], ref.eta) <= 1e-10
