"""Learned spin-up end to end (GPU): training data from the DNS, training, and
what the trained network gains over the DNS alone on held-out members.

Workload: plane Couette Re = 600, 32x49x32, minimal box; training ensemble of
64 members (the 2000-step statistics workload's seeded initial states), channel
form every 50 steps over 2000 steps (2560 pairs); network 147 -> 32 channels,
4 layers, 12 x 12 modes, BF16 matrix-core arithmetic.  Held-out members start
from states of another seed.

Gain: the network is applied 8 times (8 x 50 steps) and the DNS continues.  At
equal DNS cost h after the hand-off, the spun-up ensemble's mean and rms
profiles are compared with those of the DNS-only ensemble 400 steps later
(h + 400); the DNS-only ensemble at h is the baseline.  The spun-up members
must be closer, and the plain DNS must accept every one of them.
"""

import sys

import numpy as np
import pytest
import torch

from paper_2306_12739_amd import dns, inputs, spinup

pytestmark = pytest.mark.gpu

NAME = "couette-re600-32x49x32-e64"
GAP, SNAPS, APPS, WIN = 50, 41, 8, 100


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(E):
    w = inputs.WORKLOADS[NAME]
    e = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], E, w["dt"])
    e.set_precision(dns.PREC_MIXED_FP32)
    e.set_option(dns.OPT_GRAPH, 1)
    return e


def test_learned_spin_up_gains_over_dns_alone():
    say("case: spin-up: pairs from 64-member DNS, 8 epochs of training, 32 held-out members")
    ens = make(64)
    ens.set_state(*inputs.workload_state(NAME))
    X, Y = spinup.pairs(ens, SNAPS, GAP)
    ens.close()
    persistence = float(((X - Y).flatten(1).norm(dim=1) / Y.flatten(1).norm(dim=1)).mean())
    net = dns.SNO(channels=X.shape[1], width=32, layers=4, Mx=48, Mz=48, modes_x=12, modes_z=12,
                  max_batch=32, seed=1)
    hist = spinup.train(net, (X, Y), epochs=8, batch=32, lr=2e-3, log=say)
    say(f"persistence loss {persistence:.4f}, trained {hist[-1]:.4f}")
    assert hist[-1] < 0.9 * persistence

    held = inputs.workload_state(NAME, ensemble=32, seed=3001)
    d_s, d_0, S, rejected = spinup.gain(make, net, held, APPS, GAP, WIN, 8)
    net.close()
    say("distance to the DNS-only ensemble 400 steps ahead, per window:")
    say("  spun up :", [round(x, 3) for x in d_s])
    say("  DNS only:", [round(x, 3) for x in d_0])
    assert rejected == 0 and all(w["failed"] == 0 for w in S)
    assert max(w["div"] for w in S) <= 1e-6
    # measured: mean 0.176 vs 0.228, first window 0.208 vs 0.286
    assert np.mean(d_s) < 0.9 * np.mean(d_0)
    assert d_s[0] < 0.9 * d_0[0]
