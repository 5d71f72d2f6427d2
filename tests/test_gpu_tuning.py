"""Tile-shape variants and the tuner (GPU).

Every chunk-row variant of the advection kernel must reproduce the oracle's
de-aliased advection terms (FP64: 1e-12 relative; FP32: 2e-6 relative), and the
member tile of the per-mode kernel must not change any result bit (each output
column's contraction runs in the same order whatever columns share a tile).
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2306_12739_amd import dns, inputs

pytestmark = pytest.mark.gpu

GRIDS = [  # (flow, Re, Lx, Lz, N, Ny, dt, amplitude)
    (0, 400.0, 1.75 * np.pi, 1.2 * np.pi, 16, 33, 0.02, 0.1),
    (0, 600.0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 0.02, 0.2),
    (0, 1000.0, 1.75 * np.pi, 1.2 * np.pi, 48, 65, 0.02, 0.2),
    (1, 4200.0, 2.0 * np.pi, np.pi, 64, 97, 0.005, 0.3),
    (1, 4200.0, 2.0 * np.pi, np.pi, 72, 73, 0.005, 0.3),
    (1, 3250.0, 2.0 * np.pi, np.pi, 96, 83, 0.008, 0.3),
]
# built variants, default first: chunk rows of the general kernel, and 100 +
# chunk rows (+ 50 with the forward-z sums kept in the output buffer) of the
# lane-parallel advective kernel
ROWS = {
    dns.PREC_FP64: {16: [24, 12, 8], 32: [116, 166, 148, 198, 16, 24, 8], 48: [12, 8],
                    64: [166, 116, 16, 12, 8], 72: [12], 96: [8]},
    dns.PREC_MIXED_FP32: {16: [24, 12, 8], 32: [116, 166, 148, 198, 16, 24, 48], 48: [12, 24, 36],
                          64: [182, 116, 166, 132, 32, 24, 16], 72: [18, 12], 96: [16, 12, 8]},
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.mark.parametrize("precision", [dns.PREC_FP64, dns.PREC_MIXED_FP32])
@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: f"{g[4]}x{g[5]}")
def test_plane_variants_match_oracle(grid, precision):
    flow, Re, Lx, Lz, n, Ny, dt, amp = grid
    E = 2
    st = inputs.random_state(flow, Lx, Lz, n, Ny, n, E, amp, 2024, spectrum="k2")
    ref = oracle.OracleDNS(flow, Re, Lx, Lz, n, Ny, n, E, dt)
    ref.set_state(*st)
    rv = ref.velocities(ref.v, ref.eta, ref.U, ref.W)
    Nu, Nv, Nw, _, _ = ref.nonlinear(rv)
    tol = 1e-12 if precision == dns.PREC_FP64 else 2e-6
    ens = dns.Ensemble(flow, Re, Lx, Lz, n, Ny, n, E, dt)
    ens.set_precision(precision)
    ens.set_state(*st)
    for rows in ROWS[precision][n]:
        say(f"case: plane variant rows={rows}, grid {n}x{Ny}x{n}, precision {precision}")
        ens.set_option(dns.OPT_PLANE_ROWS, rows)
        _, nl, _ = ens.debug_stage0()
        errs = [rel(nl[i], f) for i, f in enumerate((Nu, Nv, Nw))]
        say("  errors", errs)
        assert max(errs) <= tol, (rows, errs)
    with pytest.raises(dns.DnsError):
        ens.set_option(dns.OPT_PLANE_ROWS, 7)
    ens.close()


def test_mode_tiles_bitwise_identical():
    say("case: mode member tiles 1, 2, 4, 8 on 32x49x32, E=11, 3 steps FP64")
    E = 11
    st = inputs.random_state(0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, E, 0.2, 7, spectrum="k2")
    out = []
    for et in (1, 2, 4, 8):
        ens = dns.Ensemble(0, 600.0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, E, 0.02)
        ens.set_option(dns.OPT_MODE_TILE, et)
        ens.set_state(*st)
        ens.step(3)
        out.append(ens.get_state())
        ens.close()
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b)


def test_tune_and_cache(tmp_path):
    say("case: tuner on channel 64x97x64 E=16 mixed, then from the cache")
    w = inputs.WORKLOADS["channel-re4200-64x97x64-e16"]
    cache = tmp_path / "tune.txt"
    st = inputs.workload_state("channel-re4200-64x97x64-e16")
    ens = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"],
                       w["ensemble"], w["dt"])
    ens.set_precision(dns.PREC_MIXED_FP32)
    ens.set_state(*st)
    t1 = ens.tune(str(cache))
    say("tuned:", t1)
    assert t1["plane_rows"] in ROWS[dns.PREC_MIXED_FP32][64] and not t1["from_cache"]
    assert t1["mode_members"] in (1, 2, 4, 8) and t1["plane_ms"] > 0 and t1["mode_ms"] > 0
    ens.set_option(dns.OPT_GRAPH, 1)
    ens.step(2)
    a = ens.get_state()
    ens.close()
    ens = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"],
                       w["ensemble"], w["dt"])
    ens.set_precision(dns.PREC_MIXED_FP32)
    ens.set_state(*st)
    t2 = ens.tune(str(cache))
    assert t2["from_cache"] and t2["plane_rows"] == t1["plane_rows"]
    assert t2["mode_members"] == t1["mode_members"]
    ens.set_option(dns.OPT_GRAPH, 1)
    ens.step(2)
    b = ens.get_state()
    ens.close()
    for x, y in zip(a, b):  # same tile shapes: same bits
        assert np.array_equal(x, y)
    assert len(cache.read_text().strip().splitlines()) == 1


@pytest.mark.parametrize("graph", [1, 0])
def test_member_chains_bitwise_identical(graph):
    say(f"case: member chains 1, 2, 3, 4 on 32x49x32, E=11, 3 steps, graph={graph}")
    E = 11
    st = inputs.random_state(0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, E, 0.2, 8, spectrum="k2")
    out = []
    for nc in (1, 2, 3, 4):
        ens = dns.Ensemble(0, 600.0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, E, 0.02)
        ens.set_option(dns.OPT_CHAINS, nc)
        ens.set_option(dns.OPT_GRAPH, graph)
        ens.set_option(dns.OPT_STATS, 1)
        ens.set_state(*st)
        ens.step(3)
        out.append((ens.get_state(), ens.stats()))
        ens.close()
    (ref, sref) = out[0]
    for (other, so) in out[1:]:
        for a, b in zip(ref, other):
            assert np.array_equal(a, b)
        for k in ("energy", "U", "urms", "gamma", "div_max"):
            assert np.array_equal(sref[k], so[k]), k
    with pytest.raises(dns.DnsError):
        ens = dns.Ensemble(0, 600.0, 1.75 * np.pi, 1.2 * np.pi, 32, 49, 32, 2, 0.02)
        try:
            ens.set_option(dns.OPT_CHAINS, 3)
        finally:
            ens.close()
