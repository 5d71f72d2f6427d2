"""Optimal disturbances of a streamwise-mean flow by forward-adjoint iteration
(App. B; Sec. 4, optimal-disturbance paragraph), driven over the C ABI.

Every member holds the same frozen base flow in its n_x = 0 modes
(DNS_OPT_FROZEN_MEAN) and one disturbance of a prescribed streamwise
wavenumber.  One iteration integrates the linearised equations over the
target time (DNS_OPT_QUASILINEAR = 1), reads the gains E(T)/E(0) (energy 1 at
the start), integrates the adjoint over the same time from the end states
(DNS_OPT_QUASILINEAR = 2) and orthonormalises the members in the energy norm
(dns_orthonormalize).  As in the paper the diagnostic integration uses a time
step t_f times the DNS one.

Base flow (input recipe): the paper's is a turbulent streamwise mean of its C1
case, which is not given; here laminar Couette flow plus seeded rolls and
streaks (the n_x = 0 column of a smooth random state, streak amplitude
`streak` of the wall speed) stands in for it.
"""

import argparse
import json
import time

import numpy as np

from . import dns, inputs

WORKLOAD = dict(flow=0, Re=3000.0, Lx=2.0 * np.pi, Lz=np.pi, Nx=48, Ny=63, Nz=48, dt_dns=0.008, t_f=5,
                T_opt=15.0, kx=(1, 2, 3), per_kx=15, streak=0.2, seed=1007)


def base_flow(w):
    v, eta, U, W = inputs.random_state(w["flow"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], 1, w["streak"],
                                       w["seed"], spectrum="low")
    v[:, 1:] = 0.0
    eta[:, 1:] = 0.0
    return v, eta, U, W


def initial_members(w, per_kx, kxs, base):
    bv, be, bU, bW = base
    E = per_kx * len(kxs)
    pv, pe, _, _ = inputs.random_state(w["flow"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], E, 0.1,
                                       w["seed"] + 1, spectrum="k2")
    v = np.zeros_like(pv)
    eta = np.zeros_like(pe)
    for i, kx in enumerate(kxs):
        sl = slice(i * per_kx, (i + 1) * per_kx)
        v[sl, kx] = pv[sl, kx]
        eta[sl, kx] = pe[sl, kx]
    v[:, 0] = bv[0, 0]
    eta[:, 0] = be[0, 0]
    return v, eta, np.repeat(bU, E, 0), np.repeat(bW, E, 0)


def make(w, E, precision):
    ens = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], E, w["dt_dns"] * w["t_f"])
    ens.set_precision(precision)
    ens.set_option(dns.OPT_FROZEN_MEAN, 1)
    ens.set_option(dns.OPT_GRAPH, 1)
    return ens


def iterate(ens, nsteps, iterations, tol=0.0, log=None):
    """Forward-adjoint iterations; returns the gains of the last forward run
    and the number of iterations done."""
    ens.orthonormalize()
    prev = None
    for it in range(iterations):
        ens.set_option(dns.OPT_QUASILINEAR, 1)
        ens.step(nsteps)
        gains = ens.perturbation_energy()
        ens.set_option(dns.OPT_QUASILINEAR, 2)
        ens.step(nsteps)
        ens.orthonormalize()
        if log:
            log(f"iteration {it + 1}: leading gains {np.round(np.sort(gains)[::-1][:3], 4).tolist()}")
        if prev is not None and tol > 0 and np.max(np.abs(gains - prev) / gains) < tol:
            return gains, it + 1
        prev = gains
    return gains, iterations


def main():
    ap = argparse.ArgumentParser(description="optimal disturbances, Couette C1 grid, kx/a = 1, 2, 3")
    ap.add_argument("--iterations", type=int, default=49, help="at most (49 x 2 T_opt = 1470 time units)")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--sweep", type=int, default=2, help="iterations timed per ensemble size in the sweep")
    args = ap.parse_args()
    w = dict(WORKLOAD)
    prec = dns.PREC_FP64 if args.precision == "fp64" else dns.PREC_MIXED_FP32
    nsteps = int(round(w["T_opt"] / (w["dt_dns"] * w["t_f"])))
    base = base_flow(w)
    E = w["per_kx"] * len(w["kx"])
    ens = make(w, E, prec)
    ens.set_state(*initial_members(w, w["per_kx"], w["kx"], base))
    t0 = time.perf_counter()
    gains, its = iterate(ens, nsteps, args.iterations, args.tol, log=lambda m: print(m, flush=True))
    secs = time.perf_counter() - t0
    ens.close()
    per = {int(kx): sorted(gains[i * w["per_kx"]:(i + 1) * w["per_kx"]].tolist(), reverse=True)
           for i, kx in enumerate(w["kx"])}
    # total time of one iteration against the number of disturbances computed together
    sweep = {}
    for n in (1, 3, 9, 15, 45):
        per_kx = max(1, n // len(w["kx"])) if n >= len(w["kx"]) else 1
        kxs = w["kx"] if n >= len(w["kx"]) else w["kx"][:1]
        e = make(w, per_kx * len(kxs), prec)
        e.set_state(*initial_members(w, per_kx, kxs, base))
        iterate(e, nsteps, 1)                 # warm-up (graph capture)
        t1 = time.perf_counter()
        iterate(e, nsteps, args.sweep)
        dt_it = (time.perf_counter() - t1) / args.sweep
        sweep[per_kx * len(kxs)] = {"seconds_per_iteration": dt_it,
                                    "seconds_per_iteration_per_disturbance": dt_it / (per_kx * len(kxs))}
        e.close()
        print(f"sweep: {per_kx * len(kxs)} disturbances, {dt_it:.3f} s per iteration", flush=True)
    out = {"workload": "optimal-couette-re3000-48x63x48", "precision": args.precision,
           "steps_per_integration": nsteps, "dt": w["dt_dns"] * w["t_f"], "T_opt": w["T_opt"],
           "disturbances": E, "iterations": its, "simulation_time": its * 2 * w["T_opt"],
           "seconds": secs, "seconds_per_iteration": secs / its, "gains_by_kx": per,
           "sweep": sweep}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
