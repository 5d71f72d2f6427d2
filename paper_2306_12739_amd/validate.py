"""Turbulent-statistics validation runs on the paper's resolution (72 x 73 x 72
modes on the 108 x 73 x 108 grid of its C2/P2 cases, box 2 pi x 2 x pi, dt =
0.008), driven over the C ABI.

An ensemble starts from seeded perturbations of the laminar flow and runs a
spin-up at a smaller time step on a finer wall-normal grid (the transition
from the random initial state is more violent than the developed turbulence:
at Ny = 73 it blows up within about 5 time units, at Ny = 97 it does not).  The
spun-up members are handed to the paper's grid through the channel form
(u, v, w on the 3/2 grid times Chebyshev coefficients in y, truncated to the
coarser grid's degree; dns_set_channels rebuilds admissible states), and an
ensemble at the paper's time step accumulates the one-point statistics
(Sec. 4) over windows of equal length; the friction Reynolds number Re_tau = sqrt(Re |dU/dy|_wall) of
every window shows whether the run is stationary.  The paper quotes Re_tau of
about 171 (Couette, Re = 3000) and 184 (channel).
"""

import argparse
import json
import time

import numpy as np

from . import dns, inputs


def make(w, dt, Ny=None):
    ens = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], Ny or w["Ny"], w["Nz"], w["ensemble"], dt)
    ens.set_precision(dns.PREC_MIXED_FP32)
    ens.set_option(dns.OPT_GRAPH, 1)
    return ens


def run(name, spin_steps, windows, window_steps, spin_dt, spin_ny, log=print):
    import torch
    w = inputs.WORKLOADS[name]
    ens = make(w, spin_dt, spin_ny)
    ens.set_state(*inputs.random_state(w["flow"], w["Lx"], w["Lz"], w["Nx"], spin_ny, w["Nz"], w["ensemble"],
                                       w["amplitude"], w["seed"], spectrum=w["spectrum"]))
    t0 = time.perf_counter()
    chunk = max(1, spin_steps // 10)
    for s in range(0, spin_steps, chunk):
        ens.step(min(chunk, spin_steps - s))
        st = ens.stats(allow_nonfinite=True)
        log(f"{name} spin-up step {s + chunk}: energy {st['energy'].mean():.4f}, "
            f"wall shear {0.5 * (np.abs(st['tau_lower']).mean() + np.abs(st['tau_upper']).mean()):.3e}, "
            f"failed {int(st['failed'].sum())}")
    E, P = w["ensemble"], (3 * w["Nx"] // 2) * (3 * w["Nz"] // 2)
    fine = torch.empty((E, 3 * spin_ny, P), dtype=torch.float32, device="cuda")
    ens.get_channels(fine)
    ens.close()
    Ny = w["Ny"]
    coarse = torch.stack([fine[:, f * spin_ny:f * spin_ny + Ny] for f in range(3)], dim=1)
    coarse = coarse.reshape(E, 3 * Ny, P).contiguous()
    ens = make(w, w["dt"])
    ens.set_channels(coarse)
    ens.set_option(dns.OPT_STATS, 1)
    out = []
    for k in range(windows):
        ens.stats_reset()
        ens.step(window_steps)
        st = ens.stats(allow_nonfinite=True)
        rec = {"re_tau": float(st["re_tau"]), "tau_w": float(st["tau_w"]),
               "U_center": float(st["U"][len(st["U"]) // 2]), "urms_max": float(st["urms"].max()),
               "vrms_max": float(st["vrms"].max()), "wrms_max": float(st["wrms"].max()),
               "failed": int(st["failed"].sum())}
        out.append(rec)
        log(f"{name} window {k + 1}: Re_tau {rec['re_tau']:.1f}, u'max {rec['urms_max']:.4f}")
    secs = time.perf_counter() - t0
    ens.close()
    steps = spin_steps + windows * window_steps
    return {"workload": name, "members": w["ensemble"], "dt": w["dt"], "spin_up_dt": spin_dt, "spin_up_ny": spin_ny,
            "spin_up_time": spin_steps * spin_dt,
            "window_time": window_steps * w["dt"], "windows": out,
            "re_tau_mean": float(np.mean([r["re_tau"] for r in out])),
            "seconds": secs, "ms_per_step": 1e3 * secs / steps,
            "member_steps_per_s": w["ensemble"] * steps / secs}


def main():
    ap = argparse.ArgumentParser(description="Re_tau validation at the paper's resolution")
    ap.add_argument("--workload", default="channel-re4200-72x73x72-e16")
    ap.add_argument("--spin-steps", type=int, default=25000)
    ap.add_argument("--spin-dt", type=float, default=0.004)
    ap.add_argument("--spin-ny", type=int, default=97)
    ap.add_argument("--windows", type=int, default=4)
    ap.add_argument("--window-steps", type=int, default=6250)
    args = ap.parse_args()
    out = run(args.workload, args.spin_steps, args.windows, args.window_steps, args.spin_dt, args.spin_ny,
              log=lambda m: print(m, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
