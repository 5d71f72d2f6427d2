"""Approximate S3T ensemble with stochastic forcing (Sec. 4, statistical-state-
dynamics paragraph), driven over the C ABI.

The members share one streamwise-mean flow (DNS_OPT_SHARED_MEAN), their
perturbations evolve linearised about it (DNS_OPT_QUASILINEAR), and each member
is forced independently at the streamwise wavenumber kx / a = 1 by a random
mixture of eigenvectors of the diffusion operator acting on a (Lap v, eta)
state.  Everything the time step computes runs in the HIP library; this module
prepares the forcing realizations (inputs of dns_set_forcing) and reads the
state back for diagnostics.

Forcing recipe (inputs, host side):
  * for every forced mode (n_x, n_z), the eigenpairs of the viscous operators
    of the library's own CN operators: c L = (A_v + I)^-1 (A_v - I) with
    L = Lap_D^-1 LapLap_c for v, and c Lap_D from A_eta for eta (c = dt/(2 Re));
    a v eigenvector phi forces Lap v with Lap_D phi, an eta eigenvector psi
    forces eta with psi;
  * each structure is scaled so that, taken as a velocity field, it would
    dissipate energy at the same rate (2 |mu| E / Re = 1, E its kinetic energy);
  * a realization is sum_m xi_m f_m with independent complex Gaussian xi_m of
    unit variance, redrawn every `hold` steps and scaled by 1/sqrt(hold dt)
    (piecewise-constant approximation of white noise);
  * the overall amplitude is calibrated by a short run so that the members'
    perturbation energy is `energy_ratio` times the laminar energy density.
"""

import argparse
import json
import time

import numpy as np

from . import dns, inputs

WORKLOAD = dict(flow=0, Re=1000.0, Lx=2.0 * np.pi, Lz=1.2 * np.pi, Nx=48, Ny=61, Nz=48,
                ensemble=5, dt=0.02, forced_nx=1, energy_ratio=1e-3, seed=1006)


def real_vector(p):
    """A real eigenvector from numpy's complex one (real operator, real
    eigenvalue): divide out the phase of its largest entry."""
    p = p / p[np.argmax(np.abs(p))]
    return p.real


class Forcing:
    """Diffusion-eigenvector forcing of one streamwise wavenumber."""

    def __init__(self, w, nx):
        self.w, self.nx = w, nx
        Nx, Ny, Nz = w["Nx"], w["Ny"], w["Nz"]
        L, P, NZ, N = Nx // 2, Nz // 2, Nz - 1, Ny - 2
        self.shape = (L, NZ, N)
        ops = dns.host_operators(w["flow"], w["Re"], w["Lx"], w["Lz"], Nx, Ny, Nz, w["dt"], 1)
        self.D1c, self.ccw = ops["D1c"], ops["ccw"]
        c = w["dt"] / (2.0 * w["Re"])
        eye = np.eye(N)
        kx = 2.0 * np.pi * nx / w["Lx"]
        self.modes = []  # (iz, [Lap_D phi_m] scaled, [psi_m] scaled)
        for iz in range(NZ):
            nz = iz if iz < P else iz - NZ
            kz = 2.0 * np.pi * nz / w["Lz"]
            k2 = kx * kx + kz * kz
            g = nx * P + abs(nz)
            Av, Ae = ops["ops"][g, 0], ops["ops"][g, 2]
            Lv = np.linalg.solve(Av + eye, Av - eye) / c
            Lap = np.linalg.solve(Ae + eye, Ae - eye) / c
            mu, phi = np.linalg.eig(Lv)
            lam, psi = np.linalg.eig(Lap)
            fv, fe = [], []
            for m, p in zip(mu, phi.T):
                p = real_vector(p)
                fv.append(Lap @ p * np.sqrt(w["Re"] / (2 * abs(m.real) * self.energy_v(p, k2))))
            for m, p in zip(lam, psi.T):
                p = real_vector(p)
                fe.append(p * np.sqrt(w["Re"] / (2 * abs(m.real) * self.energy_eta(p, k2))))
            self.modes.append((iz, np.stack(fv), np.stack(fe)))

    def energy_v(self, v, k2):
        """Kinetic energy density of the single-mode field with v(y) (eta = 0)."""
        full = np.zeros(len(self.ccw))
        full[1:-1] = v ** 2
        dv = self.D1c @ v
        return 0.25 * self.ccw @ (full + dv ** 2 / k2)

    def energy_eta(self, eta, k2):
        full = np.zeros(len(self.ccw))
        full[1:-1] = eta ** 2
        return 0.25 * self.ccw @ (full / k2)

    def realization(self, rng, E, scale):
        """(f_lapv, f_eta) for E members in the state layout."""
        fv = np.zeros((E,) + self.shape, complex)
        fe = np.zeros_like(fv)
        for iz, bv, be in self.modes:
            xv = (rng.standard_normal((E, bv.shape[0])) + 1j * rng.standard_normal((E, bv.shape[0]))) / np.sqrt(2)
            xe = (rng.standard_normal((E, be.shape[0])) + 1j * rng.standard_normal((E, be.shape[0]))) / np.sqrt(2)
            fv[:, self.nx, iz] = scale * (xv @ bv)
            fe[:, self.nx, iz] = scale * (xe @ be)
        return fv, fe


def mode_energy(w, D1c, ccw, v, eta):
    """Kinetic energy density per member of (a) the n_x >= 1 perturbations and
    (b) the n_x = 0, n_z != 0 part of the streamwise mean (rolls and streaks)."""
    L, P, NZ = w["Nx"] // 2, w["Nz"] // 2, w["Nz"] - 1
    nx = np.arange(L)[:, None]
    iz = np.arange(NZ)[None, :]
    nz = np.where(iz < P, iz, iz - NZ)
    k2 = (2 * np.pi * nx / w["Lx"]) ** 2 + (2 * np.pi * nz / w["Lz"]) ** 2
    k2 = np.where(k2 > 0, k2, 1.0)
    mk = np.where(nx == 0, 1.0, 2.0) * np.ones_like(k2)
    dv = np.einsum("jn,elmn->elmj", D1c, v)
    wi = ccw[1:-1]
    ev = (np.abs(v) ** 2) @ wi
    ed = (np.abs(dv) ** 2) @ ccw
    ee = (np.abs(eta) ** 2) @ wi
    dens = 0.25 * mk * (ev + (ed + ee) / k2)          # (E, L, NZ)
    pert = dens[:, 1:].sum(axis=(1, 2))
    rs = dens[:, 0, 1:].sum(axis=1)
    return pert, rs


def growth_rate(t, energy):
    """Exponential growth rate of the amplitude (sqrt of the energy) over the
    stretch before saturation: from where the energy first exceeds 1e-4 of its
    maximum to where it first exceeds 0.1 of it; None without such a stretch."""
    energy = np.asarray(energy)
    if len(energy) < 4 or not np.all(energy > 0):
        return None
    top = energy.max()
    i0 = int(np.argmax(energy > 1e-4 * top))
    i1 = int(np.argmax(energy > 0.1 * top))
    if i1 - i0 < 3:
        return None
    return float(np.polyfit(t[i0:i1], 0.5 * np.log(energy[i0:i1]), 1)[0])


def run(w, steps, cal_steps, hold, log=print):
    E = w["ensemble"]
    ens = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], E, w["dt"])
    ens.set_precision(dns.PREC_MIXED_FP32)
    ens.set_option(dns.OPT_SHARED_MEAN, 1)
    ens.set_option(dns.OPT_QUASILINEAR, 1)
    ens.set_option(dns.OPT_GRAPH, 1)
    v, eta, U, W = inputs.random_state(w["flow"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], E, 0.0,
                                       w["seed"])
    ens.set_state(v, eta, U, W)
    forcing = Forcing(w, w["forced_nx"])
    rng = np.random.default_rng(w["seed"])
    lam_energy = 1.0 / 6.0   # (1/Ly) int U^2 / 2 dy of laminar Couette U = y
    target = w["energy_ratio"] * lam_energy

    def advance(nsteps, amp, record_every=0):
        rec = []
        t0 = time.perf_counter()
        for s in range(0, nsteps, hold):
            fv, fe = forcing.realization(rng, E, amp / np.sqrt(hold * w["dt"]))
            ens.set_forcing(fv, fe)
            ens.step(min(hold, nsteps - s))
            if record_every and (s // hold) % (record_every // hold) == 0:
                vv, ee, _, _ = ens.get_state()
                pert, rs = mode_energy(w, forcing.D1c, forcing.ccw, vv, ee)
                rec.append((s + hold, float(pert.mean()), float(rs[0])))
                if len(rec) % 10 == 0:
                    log(f"step {s + hold}: perturbation energy {rec[-1][1]:.3e}, roll-streak energy {rec[-1][2]:.3e}")
        ens.sync()
        return rec, time.perf_counter() - t0

    # calibration at a weak amplitude (the mean stays laminar to O(amp^2)): the
    # quasi-linear perturbation energy is then quadratic in the amplitude
    amp0 = 1e-6
    rec, _ = advance(cal_steps, amp0, record_every=max(hold, cal_steps // 20))
    late = [r[1] for r in rec[len(rec) // 2:]]
    amp = amp0 * np.sqrt(target / np.mean(late))
    log(f"calibrated forcing amplitude {amp:.4e} (perturbation energy {np.mean(late):.3e} at {amp0})")
    ens.set_state(v, eta, U, W)
    rec, secs = advance(steps, amp, record_every=max(hold, steps // 200))
    s = ens.stats(allow_nonfinite=True)
    # step rate of the library alone (forcing held, no host work in between)
    ens.step(20)
    ens.sync()
    t0 = time.perf_counter()
    ens.step(1000)
    ens.sync()
    device_ms = (time.perf_counter() - t0)  # seconds per 1000 steps = ms per step
    plane_ms, mode_ms = ens.kernel_times(10)
    ens.set_option(dns.OPT_QUASILINEAR, 0)
    plane_ms_full, _ = ens.kernel_times(10)
    ens.close()
    t = np.array([r[0] for r in rec]) * w["dt"]
    pert = np.array([r[1] for r in rec])
    rs = np.array([r[2] for r in rec])
    half = len(t) // 2
    sigma = growth_rate(t, rs)
    return {"workload": "s3t-couette-re1000-48x61x48-e5", "members": E, "steps": steps,
            "hold_steps": hold, "seconds": secs, "ms_per_step_with_forcing_updates": 1e3 * secs / steps,
            "ms_per_step": device_ms, "member_steps_per_s_library": E * 1000 / device_ms,
            "member_steps_per_s": E * steps / secs, "forcing_amplitude": amp,
            "perturbation_energy_over_laminar": float(pert[half:].mean() / lam_energy),
            "roll_streak_energy": rs.tolist(), "time": t.tolist(),
            "roll_streak_amplitude_growth_rate": sigma, "failed": int(s["failed"].sum()),
            "plane_kernel_ms_quasilinear": plane_ms, "plane_kernel_ms_full_advection": plane_ms_full,
            "mode_kernel_ms": mode_ms}


def main():
    ap = argparse.ArgumentParser(description="approximate S3T ensemble, Couette Re=1000, 48x61x48, 5 members")
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--calibration-steps", type=int, default=7500)
    ap.add_argument("--hold", type=int, default=5)
    args = ap.parse_args()
    out = run(dict(WORKLOAD), args.steps, args.calibration_steps, args.hold, log=lambda m: print(m, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
