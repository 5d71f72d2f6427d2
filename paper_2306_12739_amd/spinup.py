"""Learned spin-up of ensemble members over the C ABI (include/sno.h).

Three stages, each a thin sequence of library calls (every arithmetic step runs
in the HIP library; torch only holds device memory):
  * pairs()   -- run a DNS ensemble and take its channel form every ``gap``
                 steps; consecutive snapshots of a member form (input, target)
                 pairs; transient_pairs() repeats this from fresh initial
                 states so that the pairs sample the transient the network is
                 meant to replace;
  * train()   -- AdamW on the relative-L2 loss over contiguous mini-batches
                 in a seeded random order, with a cosine learning-rate decay;
  * spin_up() -- apply the network ``applications`` times to members' channel
                 form and rebuild admissible states from the prediction; the
                 DNS then continues and checks every member.
"""

import argparse
import json
import math
import time

import numpy as np
import torch

from . import dns, inputs


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


def transient_pairs(make, rounds, snapshots, gap, members, state_of_seed, seed0):
    """Pairs from ``rounds`` ensembles of fresh initial states (seeds seed0 + r).

    Returns a list of (X, Y) blocks, one per round."""
    blocks = []
    for r in range(rounds):
        ens = make(members)
        ens.set_state(*state_of_seed(seed0 + r))
        blocks.append(pairs(ens, snapshots, gap))
        ens.close()
    return blocks


def train(net, data, epochs, batch, lr=2e-3, lr_final=1e-4, weight_decay=1e-4, seed=0, log=None):
    """Train on contiguous mini-batches in a seeded random order.

    data: an (X, Y) pair or a list of them.  Returns the mean loss of each epoch."""
    blocks = [data] if isinstance(data, tuple) else list(data)
    starts = [(b, s0) for b, (X, _) in enumerate(blocks) for s0 in range(0, X.shape[0] - batch + 1, batch)]
    rng = np.random.default_rng(seed)
    total = epochs * len(starts)
    it = 0
    history = []
    for ep in range(epochs):
        losses = []
        for i in rng.permutation(len(starts)):
            b, s0 = starts[i]
            X, Y = blocks[b]
            frac = it / max(total - 1, 1)
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
            losses.append(net.train_step(X[s0:s0 + batch], Y[s0:s0 + batch], lr=rate,
                                         weight_decay=weight_decay))
            it += 1
        history.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: loss {history[-1]:.5f}")
    return history


def spin_up(ens, net, applications, member0=0, count=None, check_steps=0):
    """Advance members [member0, member0 + count) by ``applications`` network
    steps and hand the admissible states back to the DNS.

    check_steps > 0: the DNS then runs ``check_steps`` steps; members it flags non-finite
    get their original state back and re-run those steps as plain DNS
    members.  Returns the number of members the DNS rejected."""
    count = ens.E - member0 if count is None else count
    original = ens.get_state(member0, count) if check_steps else None
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
    if not check_steps:
        return 0
    before = ens.get_state()
    ens.step(check_steps)
    failed = ens.stats(allow_nonfinite=True)["failed"][member0:member0 + count].astype(bool)
    if not failed.any():
        return 0
    # put rejected members back to their original states; every other member
    # returns to its hand-off state, so that all members restart together
    v, eta, U, W = (a.copy() for a in before)
    for i in np.nonzero(failed)[0]:
        m = member0 + i
        v[m], eta[m], U[m], W[m] = (o[i] for o in original)
    ens.set_state(v, eta, U, W)
    ens.step(check_steps)
    return int(failed.sum())


def profile_windows(ens, n, win):
    """Mean and rms profiles over n consecutive windows of ``win`` steps."""
    ens.set_option(dns.OPT_STATS, 1)
    out = []
    for _ in range(n):
        ens.stats_reset()
        ens.step(win)
        s = ens.stats()
        out.append({k: s[k].copy() for k in ("U", "urms", "vrms", "wrms")}
                   | {"div": float(s["div_max"].max()), "failed": int(s["failed"].sum())})
    return out


def profile_distance(a, b):
    """Mean over U, u', v', w' of the relative 2-norm distance of the profiles."""
    return float(np.mean([np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k])
                          for k in ("U", "urms", "vrms", "wrms")]))


def gain(make, net, held, applications, gap, win, windows, check_steps=0):
    """Spun-up vs DNS-only ensembles of the same held-out initial states.

    Returns the per-window distances of the spun-up ensemble (after the
    hand-off) and of the DNS-only ensemble at equal DNS cost, both measured
    against the DNS-only ensemble ``applications * gap`` steps ahead."""
    skip = applications * gap // win
    ref = make(held[0].shape[0])
    ref.set_state(*held)
    R = profile_windows(ref, windows + skip, win)
    ref.close()
    arm = make(held[0].shape[0])
    arm.set_state(*held)
    rejected = spin_up(arm, net, applications, check_steps=check_steps)
    S = profile_windows(arm, windows, win)
    arm.close()
    d_s = [profile_distance(S[h], R[h + skip]) for h in range(windows)]
    d_0 = [profile_distance(R[h], R[h + skip]) for h in range(windows)]
    return d_s, d_0, S, rejected


def main():
    ap = argparse.ArgumentParser(description="learned spin-up on the Couette Re=600 32x49x32 ensemble")
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--snapshots", type=int, default=17, help="per fresh ensemble (the transient)")
    ap.add_argument("--gap", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--applications", type=int, default=8)
    ap.add_argument("--held-out", type=int, default=64)
    ap.add_argument("--window", type=int, default=100, help="DNS steps per statistics window")
    ap.add_argument("--windows", type=int, default=20,
                    help="windows of DNS continuation after the hand-off (20 x 100 = 2000 steps)")
    args = ap.parse_args()
    name = "couette-re600-32x49x32-e64"
    w = inputs.WORKLOADS[name]

    def make(E):
        e = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], E, w["dt"])
        e.set_precision(dns.PREC_MIXED_FP32)
        e.set_option(dns.OPT_GRAPH, 1)
        return e

    E = w["ensemble"]
    per_round = E * (args.snapshots - 1)
    rounds = -(-args.pairs // per_round)
    t0 = time.perf_counter()
    blocks = transient_pairs(make, rounds, args.snapshots, args.gap, E,
                             lambda sd: inputs.workload_state(name, seed=sd), w["seed"])
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    npairs = sum(X.shape[0] for X, _ in blocks)
    persistence = float(np.mean([float(((X - Y).flatten(1).norm(dim=1) / Y.flatten(1).norm(dim=1)).mean())
                                 for X, Y in blocks]))
    print(f"{npairs} pairs from {rounds} fresh ensembles in {t_data:.1f} s; persistence loss {persistence:.4f}",
          flush=True)
    net = dns.SNO(channels=blocks[0][0].shape[1], width=32, layers=4, Mx=48, Mz=48, modes_x=12, modes_z=12,
                  max_batch=args.batch, seed=1)
    t0 = time.perf_counter()
    hist = train(net, blocks, args.epochs, args.batch, lr=args.lr, log=lambda m: print(m, flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = args.epochs * sum(X.shape[0] // args.batch for X, _ in blocks)
    del blocks
    torch.cuda.empty_cache()
    held = inputs.workload_state(name, ensemble=args.held_out, seed=3001)
    t0 = time.perf_counter()
    d_s, d_0, S, rejected = gain(make, net, held, args.applications, args.gap, args.window, args.windows,
                                 check_steps=50)
    t_gain = time.perf_counter() - t0
    out = {"pairs": npairs, "rounds": rounds, "dns_steps_for_data": rounds * (args.snapshots - 1) * args.gap,
           "data_seconds": t_data, "persistence_loss": persistence, "epoch_loss": hist,
           "train_seconds": t_train, "train_steps": steps, "train_samples_per_s": steps * args.batch / t_train,
           "applications": args.applications, "held_out": args.held_out,
           "continuation_steps": args.window * args.windows, "window_steps": args.window,
           "gain_seconds": t_gain,
           "distance_spun_up": d_s, "distance_dns_only": d_0,
           "mean_distance_spun_up": float(np.mean(d_s)), "mean_distance_dns_only": float(np.mean(d_0)),
           "rejected_by_dns": rejected, "failed_members": sum(x["failed"] for x in S),
           "div_max": max(x["div"] for x in S)}
    print(json.dumps(out), flush=True)
    net.close()


if __name__ == "__main__":
    main()
