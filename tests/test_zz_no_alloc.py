"""Allocation-free hand-off of channel-form states (dns_set_channels_noalloc)
against the allocating dns_set_channels: the same members end in bitwise the
same states, on two calls in a row (the second with fewer members and other
data), step on identically afterwards, and a count whose intermediates exceed
the fixed scratch is rejected without touching the state."""

import sys

import numpy as np
import pytest
import torch

from paper_2306_12739_amd import dns, inputs

pytestmark = pytest.mark.gpu

BOX = (1.75 * np.pi, 1.2 * np.pi)
N, NY, E = 32, 49, 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(st):
    ens = dns.Ensemble(0, 600.0, BOX[0], BOX[1], N, NY, N, E, 0.02)
    ens.set_state(*st)
    return ens


def same_state(a, b):
    for name, x, y in zip(("v", "eta", "U", "W"), a.get_state(), b.get_state()):
        assert np.array_equal(x, y), name


def test_noalloc_set_channels_matches_set_channels():
    say(f"case: dns_set_channels_noalloc vs dns_set_channels, {N}x{NY}x{N}, {E} members")
    st = inputs.random_state(0, BOX[0], BOX[1], N, NY, N, E, 0.2, 41, spectrum="k2")
    src = make(st)
    src.step(3)
    chans = torch.zeros((E, 3 * NY, (3 * N // 2) ** 2), dtype=torch.float32, device="cuda")
    src.get_channels(chans)
    torch.cuda.synchronize()
    src.close()

    ref, got = make(st), make(st)
    # first call: 16 members [2, 18) from channels of members 0..15
    ref.set_channels(chans[0:16], member0=2)
    got.set_channels_noalloc(chans[0:16], member0=2)
    same_state(ref, got)
    v0 = got.get_state()[0]
    assert not np.array_equal(v0[2:18], st[0][2:18])   # the hand-off did replace them
    assert np.array_equal(v0[:2], st[0][:2]) and np.array_equal(v0[18:], st[0][18:])
    say("  first call (16 members): bitwise equal")

    # second call, smaller and with other data: members [5, 8) from channels 17..19
    ref.set_channels(chans[17:20], member0=5)
    got.set_channels_noalloc(chans[17:20], member0=5)
    same_state(ref, got)
    say("  second call (3 members): bitwise equal")

    # both continue identically, no member flagged
    ref.step(2)
    got.step(2)
    same_state(ref, got)
    assert not ref.stats()["failed"].any() and not got.stats()["failed"].any()
    say("  two steps after the hand-offs: bitwise equal")

    # a count whose intermediates exceed the scratch is refused, state untouched
    per_member = 3 * NY * ((3 * N // 2) ** 2 + 2 * (N // 2) * (N - 1)) * 8
    limit = (64 << 20) // per_member
    assert limit < E
    before = got.get_state()
    with pytest.raises(dns.DnsError) as info:
        got.set_channels_noalloc(chans[0:limit + 1], member0=0)
    assert info.value.code == dns.DNS_E_INVALID and f"at most {limit} members" in str(info.value)
    for x, y in zip(before, got.get_state()):
        assert np.array_equal(x, y)
    say(f"  {limit + 1} members refused (limit {limit})")
    ref.close()
    got.close()
