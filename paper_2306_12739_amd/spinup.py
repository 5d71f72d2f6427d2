"""Learned spin-up of ensemble members over the C ABI (include/sno.h).

Three stages, each a thin sequence of library calls (every arithmetic step runs
in the HIP library; torch only holds device memory):
  * pairs()   -- run a DNS ensemble and take its channel form every ``gap``
                 steps; consecutive snapshots of a member form (input, target)
                 pairs;
  * train()   -- AdamW on the relative-L2 loss over contiguous mini-batches
                 in a seeded random order, with a cosine learning-rate decay;
  * spin_up() -- apply the network ``applications`` times to members' channel
                 form and rebuild admissible states from the prediction; the
                 DNS then continues and judges every member.
"""

import math

import numpy as np
import torch

from . import dns


def channel_shape(ens):
    return 3 * ens.Ny, (3 * ens.Nx // 2) * (3 * ens.Nz // 2)


def pairs(ens, snapshots, gap):
    """Channel-form snapshots of every member, ``gap`` steps apart.

    Returns (X, Y): device float32 views of shape ((snapshots - 1) E, C, P);
    sample s E + e pairs member e at snapshot s with the same member at s + 1.
    """
    C, P = channel_shape(ens)
    snaps = torch.empty((snapshots, ens.E, C, P), dtype=torch.float32, device="cuda")
    for s in range(snapshots):
        if s:
            ens.step(gap)
        ens.get_channels(snaps[s])
    X = snaps[:-1].reshape(-1, C, P)
    Y = snaps[1:].reshape(-1, C, P)
    return X, Y


def train(net, X, Y, epochs, batch, lr=2e-3, lr_final=1e-4, weight_decay=1e-4, seed=0, log=None):
    """Train on contiguous mini-batches of (X, Y) in a seeded random order.

    Returns the mean loss of each epoch."""
    n = X.shape[0]
    starts = np.arange(0, n - batch + 1, batch)
    rng = np.random.default_rng(seed)
    total = epochs * len(starts)
    it = 0
    history = []
    for ep in range(epochs):
        losses = []
        for s0 in rng.permutation(starts):
            frac = it / max(total - 1, 1)
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
            losses.append(net.train_step(X[s0:s0 + batch], Y[s0:s0 + batch], lr=rate,
                                         weight_decay=weight_decay))
            it += 1
        history.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: loss {history[-1]:.5f}")
    return history


def spin_up(ens, net, applications, member0=0, count=None):
    """Advance members [member0, member0 + count) by ``applications`` network
    steps and hand the admissible states back to the DNS."""
    count = ens.E - member0 if count is None else count
    C, P = channel_shape(ens)
    x = torch.empty((count, C, P), dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ens.get_channels(x, member0)
    cap = net.cfg.max_batch
    for _ in range(applications):
        for b0 in range(0, count, cap):
            b1 = min(count, b0 + cap)
            net.forward(x[b0:b1], y[b0:b1])
        x, y = y, x
    net.sync()
    ens.set_channels(x, member0)
    return x
