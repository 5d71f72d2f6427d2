"""GPU parity of the Helmholtz-Poisson (KMM) v discretization against the
oracle's, through the C ABI (the operators change; the kernels do not).

Bars: states 1e-10 relative per field after 100 FP64 steps (Couette) and 10
steps (channel, ragged member tiles); mixed precision 1e-4 after 100 steps;
switching back to the clamped operator reproduces a clamped run bitwise.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2306_12739_amd import dns, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def errors(gpu, ref):
    v, eta, U, W = gpu.get_state()
    lam = ref.laminar_profile()[None, :]
    return {"v": rel(v, ref.v), "eta": rel(eta, ref.eta), "U-Ulam": rel(U - lam, ref.U - lam)}


@pytest.mark.parametrize("precision", [dns.PREC_FP64, dns.PREC_MIXED_FP32])
def test_kmm_couette_100_steps(precision):
    say(f"case: KMM v discretization, couette 16x33x16 E=2, 100 steps, precision {precision}")
    w = inputs.WORKLOADS["couette-re400-16x33x16-e2"]
    st = inputs.workload_state("couette-re400-16x33x16-e2")
    gpu = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], 2, w["dt"])
    gpu.set_option(dns.OPT_V_DISCRETIZATION, dns.VDISC_KMM)
    gpu.set_precision(precision)
    gpu.set_state(*st)
    ref = oracle.OracleDNS(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], 2, w["dt"],
                           v_discretization="kmm")
    ref.set_state(*st)
    gpu.step(100)
    ref.step(100)
    errs = errors(gpu, ref)
    say("errors:", errs)
    bar = 1e-10 if precision == dns.PREC_FP64 else 1e-4
    for k, e in errs.items():
        assert e <= bar, (k, e)
    gpu.close()


def test_kmm_channel_ragged_members_fp64():
    say("case: KMM v discretization, channel 32x49x32 Re=2000 E=5 FP64, 10 steps dt=0.01")
    st = inputs.random_state(1, 2 * np.pi, np.pi, 32, 49, 32, 5, 0.3, 51, spectrum="k2")
    gpu = dns.Ensemble(1, 2000.0, 2 * np.pi, np.pi, 32, 49, 32, 5, 0.01)
    gpu.set_option(dns.OPT_V_DISCRETIZATION, dns.VDISC_KMM)
    gpu.set_state(*st)
    ref = oracle.OracleDNS(1, 2000.0, 2 * np.pi, np.pi, 32, 49, 32, 5, 0.01, v_discretization="kmm")
    ref.set_state(*st)
    gpu.step(10)
    ref.step(10)
    errs = errors(gpu, ref)
    say("errors:", errs)
    for k, e in errs.items():
        assert e <= 1e-10, (k, e)
    np.testing.assert_allclose(gpu.stats()["flux"], 4.0 / 3.0, rtol=1e-13)
    gpu.close()


def test_switching_back_restores_the_clamped_operator_bitwise():
    say("case: clamped -> KMM -> clamped operators, graph on, couette 32x49x32 E=3")
    st = inputs.random_state(0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, 3, 0.2, 52, spectrum="k2")
    out = []
    for switch in (False, True):
        ens = dns.Ensemble(0, 600.0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, 3, 0.02)
        ens.set_option(dns.OPT_GRAPH, 1)
        ens.set_state(*st)
        ens.step(1)
        if switch:
            ens.set_option(dns.OPT_V_DISCRETIZATION, dns.VDISC_KMM)
            ens.set_option(dns.OPT_V_DISCRETIZATION, dns.VDISC_CLAMPED)
        ens.step(2)
        out.append(ens.get_state())
        with pytest.raises(dns.DnsError):
            ens.set_option(dns.OPT_V_DISCRETIZATION, 2)
        ens.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)
