"""Throughput benchmark of the ensemble CN/RK3 step on one MI355X.

One "step" is one full time step (three RK3 sub-steps: advection stage, right-
hand sides, CN solves, velocity recovery, diagnostics) of every member of the
ensemble, on synthetic seeded initial conditions already resident in HBM.

Default workload: plane Poiseuille flow at constant flux, Re = 4200 (laminar
centreline; bulk Re 5600, the Re_tau ~ 180 case), box 2pi x 2 x pi,
64 x 97 x 64 modes/points, 16 members, dt = 0.005, mixed precision (x-z FFTs,
advection products and the stage buffers between the two kernels in FP32;
y-derivative products, implicit solves, mean flow and flux update in FP64),
each step replayed as one hipGraph.

Prints ONE JSON line with member-steps/s, the same ensemble's FP64 step and
the mixed/FP64 speed-up, the roofline fraction of the dominant kernel (timed
live with HIP events on the library's stream), and the CPU oracle timed on
this host as a reported baseline.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector ALU peak: 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz.  Packed
# FP32 instructions are disabled at compile time, so FP32 and FP64 vector peaks are equal.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# published dense FP64 matrix-core rate of the MI355X
FP64_MATRIX_TFLOPS = 78.6
# The published FP32 vector figure counts packed (two-wide) FP32 FMAs.
FP32_PUBLISHED_TFLOPS = 157.3
METRIC = "ensemble member-steps/s at Re_tau~180; mixed vs FP64 at <=1% stats error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["mixed", "fp64", "3xbf16", "fp32mm"], default="mixed")
    ap.add_argument("--workload", default="channel-re4200-64x97x64-e16")
    ap.add_argument("--ensemble", type=int, default=None)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tile shapes instead of running the tuner first")
    ap.add_argument("--tune-cache", default=None,
                    help="tuner cache file: a tiling found there is applied without timing and new "
                         "results are appended, so that several runs (profiler passes) use one choice")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--advection", choices=["advective", "rotational"], default="advective",
                    help="form of the nonlinear term for the headline run; the other form is "
                         "timed briefly on the same ensemble and reported beside it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--steps-only", action="store_true",
                    help="time the headline steps only and print the line without the per-kernel, "
                         "FP64, other-form, serial and CPU figures (for kernel traces whose last "
                         "dispatches are the timed steps)")
    return ap.parse_args()


def kernel_model(w, E, precision, form="advective"):
    """Algorithmic bytes and flops of one launch of each hot kernel."""
    Nx, Ny, Nz = w["Nx"], w["Ny"], w["Nz"]
    L, P, NZ, My, N = Nx // 2, Nz // 2, Nz - 1, Ny, Ny - 2
    K, G = L * NZ, L * P
    Mx, Mz = 3 * L, 3 * P
    vt = 8 if precision == "fp64" else 4
    cplx = 2 * vt
    # advection kernel, in the launch shape of a step (the My - 2 interior
    # planes): read u,v,w,uy,wy spectra, write Nu,Nv,Nw spectra, plane means
    Mp = My - 2
    plane_bytes = (5 + 3) * Mp * K * E * cplx + 2 * Mp * E * 8
    # flops: complex FFT 5 n log2 n, real FFT 2.5 n log2 n (conventional counts);
    # advective form: 8 z- and 11 x-inverses, u.grad u and the means; rotational
    # form: 6 and 6, omega x u and the means
    nz_inv, nx_inv, pw = (6, 6, 9 + 4) if form == "rotational" else (8, 11, 3 * 5 + 2 * 2)
    zinv = nz_inv * L * 5 * Mz * np.log2(Mz)
    xinv = nx_inv * Mz * 2.5 * Mx * np.log2(Mx)
    prod = Mx * Mz * pw
    xfwd = 3 * Mz * 2.5 * Mx * np.log2(Mx)
    zfwd = 3 * L * 5 * Mz * np.log2(Mz)
    plane_flops = (zinv + xinv + prod + xfwd + zfwd) * Mp * E
    # per-(kx,kz) kernel (second sub-step): N spectra in, velocity spectra out,
    # state in and history in/out in FP64, and the y-parity halves of
    # [A_v | B_v] and [A_eta | B_eta] once per group
    He, Ho = (N + 1) // 2, N // 2
    Fe, Fo = He + 1, Ho + 1
    op_words = 2 * (He * 2 * He + Ho * 2 * Ho)
    mode_bytes = (3 + 5) * My * K * E * cplx + 2 * K * N * E * 16 + 2 * 2 * K * N * E * 16 \
        + G * op_words * 8
    cols = 2 * K * E  # real columns over all modes
    macs = 2 * (2 * He * He + 2 * Ho * Ho) + (Ho * Fe + He * Fo) + (Fo * He + Fe * Ho) \
        + 2 * 2 * Fe * Fo
    mode_flops = cols * 2 * macs
    return {"plane": (plane_bytes, plane_flops), "mode": (mode_bytes, mode_flops)}


def source_hash(files):
    """Hash of the named files under paper_2306_12739_amd/csrc (the sources of
    one kernel), in the order given."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_12739_amd", "csrc")
    for f in files:
        p = os.path.join(csrc, f)
        if not os.path.exists(p):
            return None
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch from the committed rocprofv3 counter record, only
    if it was taken on the current sources of that kernel."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    rec = d.get("kernels", {}).get(f"{kernel}/{workload}/{precision}")
    if rec is None or rec.get("source_hash") != source_hash(rec.get("sources", [])):
        return None
    return rec.get("bytes_per_launch")


def host_cpu():
    """CPU model and counts as lscpu reports them, plus the family/model/stepping
    numbers of /proc/cpuinfo (a virtualised host may print a generic name)."""
    info = {}
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in txt.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket",
                             "Socket(s)", "CPU family", "Model", "Stepping", "CPU max MHz"):
                info[k.strip()] = v.strip()
    except Exception:
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    return info


def cpu_baseline(w, name):
    """The oracle as it stands, on this host: every member of the workload for
    3 steps (operators built before the timed region)."""
    import oracle
    from paper_2306_12739_amd import inputs
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count()
    members, steps = w["ensemble"], 3
    sim = oracle.OracleDNS(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"],
                           members, w["dt"])
    sim.set_state(*inputs.workload_state(name, ensemble=members))
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    # a smaller sample on one host thread (2 members x 3 steps)
    one = None
    try:
        from threadpoolctl import threadpool_limits
        small = oracle.OracleDNS(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], 2, w["dt"])
        small.set_state(*inputs.workload_state(name, ensemble=2))
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            small.step(steps)
            one = 2 * steps / (time.perf_counter() - t1)
    except ImportError:
        pass
    # the smaller workloads: the 2-member Couette case run fully, one step of all
    # 64 members of the 32x49x32 case (same threads)
    others = {}
    for oname, E, nsteps in (("couette-re400-16x33x16-e2", 2, 100), ("couette-re600-32x49x32-e64", 64, 1)):
        ow = inputs.WORKLOADS[oname]
        osim = oracle.OracleDNS(ow["flow"], ow["Re"], ow["Lx"], ow["Lz"], ow["Nx"], ow["Ny"], ow["Nz"], E,
                                ow["dt"])
        osim.set_state(*inputs.workload_state(oname, ensemble=E))
        t1 = time.perf_counter()
        osim.step(nsteps)
        others[oname] = {"member_steps_per_s": E * nsteps / (time.perf_counter() - t1),
                         "sample": f"{E} members x {nsteps} steps"}
    cpu = host_cpu()
    return {"value": members * steps / dt, "unit": "member-steps/s", "cores": int(cores),
            "kind": "oracle", "cpu_model": cpu.get("Model name"), "host": cpu,
            "value_1_thread": one, "sample_1_thread": f"2 members x {steps} steps",
            "sample": f"all {members} members x {steps} steps of {name} (numpy FP64, operators prebuilt)",
            "other_workloads": others}


def serial_gpu(w, precision, stream, steps=50):
    """One member at a time on the GPU (the paper's serial-versus-vectorized
    comparison): member-steps/s of a one-member ensemble."""
    from paper_2306_12739_amd import dns, inputs
    import torch
    one = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], 1, w["dt"])
    one.set_stream(stream)
    one.set_precision(precision)
    one.set_option(dns.OPT_GRAPH, 1)
    st = inputs.random_state(w["flow"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], 1, w["amplitude"],
                             w["seed"], spectrum=w["spectrum"])
    one.set_state(*st)
    one.step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    one.close()
    return steps / dt


def time_steps(ens, stream, warmup, steps):
    import torch
    ens.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    ens.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (the ensemble shards by members across GPUs "
              f"with no exchange; a multi-GPU run is not built here). Got --gpus {args.gpus}.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2306_12739_amd import dns, inputs

    name = args.workload
    w = inputs.WORKLOADS[name]
    E = args.ensemble or w["ensemble"]
    torch.cuda.set_device(0)
    # a dedicated stream (default priority): the library launches on it and the
    # timing events are recorded on it
    stream = torch.cuda.Stream()
    ens = dns.Ensemble(w["flow"], w["Re"], w["Lx"], w["Lz"], w["Nx"], w["Ny"], w["Nz"], E, w["dt"])
    ens.set_stream(stream)
    ens_precision = {"fp64": dns.PREC_FP64, "mixed": dns.PREC_MIXED_FP32,
                     "3xbf16": dns.PREC_MIXED_3XBF16, "fp32mm": dns.PREC_MIXED_FP32MM}[args.precision]
    ens.set_precision(ens_precision)
    ens.set_option(dns.OPT_GRAPH, 0 if args.no_graph else 1)
    forms = {"advective": dns.ADV_ADVECTIVE, "rotational": dns.ADV_ROTATIONAL}
    ens.set_advection(forms[args.advection])
    ens.set_state(*inputs.workload_state(name, ensemble=E))
    tuning = None if args.no_tune else ens.tune(args.tune_cache)

    ens.step(args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    ens.step(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    if abs(ms / 1e3 - wall) > 0.2 * wall + 0.05:
        print(f"warning: event time {ms / 1e3:.3f}s vs wall {wall:.3f}s", file=sys.stderr)
    s = ens.stats(allow_nonfinite=True)
    if s["rc"] != 0:
        print(f"warning: {int(s['failed'].sum())} members non-finite", file=sys.stderr)
    if args.steps_only:
        ens.close()
        print(json.dumps({"metric": METRIC, "value": E * args.steps / (ms / 1e3), "unit": "member-steps/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": ms / args.steps, "steps_only": True, "tuning": tuning}), flush=True)
        return

    plane_ms, mode_ms = ens.kernel_times(args.kernel_reps)
    # the other advection form, briefly, on the same ensemble (tuned for itself)
    other = "rotational" if args.advection == "advective" else "advective"
    ens.set_advection(forms[other])
    ens.set_state(*inputs.workload_state(name, ensemble=E))
    if not args.no_tune:
        ens.tune(args.tune_cache)
    o_steps = max(20, args.steps // 4)
    o_ms = time_steps(ens, stream, 10, o_steps)
    o_plane_ms, _ = ens.kernel_times(args.kernel_reps)
    o_model = kernel_model(w, E, args.precision, other)["plane"]
    alternative = {"advection": other, "steps": o_steps, "ms_per_step": o_ms / o_steps,
                   "value": E * o_steps / (o_ms / 1e3), "plane_ms": o_plane_ms,
                   "plane_TFLOP/s": o_model[1] / (o_plane_ms * 1e-3) / 1e12}
    # the plain FP64 GPU step of the same ensemble (tuned for itself)
    fp64 = None
    if args.precision != "fp64":
        ens.set_advection(forms[args.advection])
        ens.set_precision(dns.PREC_FP64)
        ens.set_state(*inputs.workload_state(name, ensemble=E))
        if not args.no_tune:
            ens.tune(args.tune_cache)
        f_steps = max(20, args.steps // 2)
        f_ms = time_steps(ens, stream, 5, f_steps)
        fp64 = {"steps": f_steps, "ms_per_step": f_ms / f_steps, "value": E * f_steps / (f_ms / 1e3)}
        fp64["speedup_of_headline"] = fp64["ms_per_step"] / (ms / args.steps)
        ens.set_precision(ens_precision)
    serial = serial_gpu(w, ens_precision, stream)
    if args.copy_calibration:
        # reference kernel of known traffic: reads and writes exactly 256 MiB
        with torch.cuda.stream(stream):
            src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            dst.copy_(src)
        torch.cuda.synchronize()
    ens.close()

    ms_step = ms / args.steps
    value = E * args.steps / (ms / 1e3)
    gp_paper = (w["Nx"] - 1) * (w["Nz"] - 1) * (w["Ny"] - 2)
    model = kernel_model(w, E, args.precision, args.advection)
    per_kernel = {}
    for k, t in (("plane", plane_ms), ("mode", mode_ms)):
        b, f = model[k]
        per_kernel[k] = {"ms": t, "GB/s": b / (t * 1e-3) / 1e9, "TFLOP/s": f / (t * 1e-3) / 1e12,
                         "alg_bytes": b, "alg_flops": f,
                         "traffic": measured_traffic(k, name, args.precision)
                         if args.advection == "advective" else None}
    # each kernel against its own roof: the advection kernel is bound by vector-ALU issue
    # (FFT and product flops against the non-packed vector rate), the per-mode kernel by HBM
    # (its algorithmic bytes; its FP64 matrix work needs less time at peak)
    per_kernel["plane"]["frac_valu"] = per_kernel["plane"]["TFLOP/s"] / VALU_PEAK_TFLOPS
    per_kernel["mode"]["frac_hbm"] = per_kernel["mode"]["GB/s"] / HBM_PEAK_GBS
    per_kernel["mode"]["frac_fp64_matrix"] = per_kernel["mode"]["TFLOP/s"] / FP64_MATRIX_TFLOPS
    dom = "plane" if plane_ms >= mode_ms else "mode"
    pk = per_kernel[dom]
    if dom == "plane":
        roof = {"bound": "alu", "achieved": pk["TFLOP/s"], "peak": VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": pk["TFLOP/s"] / VALU_PEAK_TFLOPS,
                "peak_published": FP32_PUBLISHED_TFLOPS,
                "frac_published": pk["TFLOP/s"] / FP32_PUBLISHED_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": pk["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": pk["GB/s"] / HBM_PEAK_GBS}
    roof["kernel"] = dom
    roof["traffic"] = measured_traffic(dom, name, args.precision) if args.advection == "advective" else None

    cpu = None if args.no_cpu_baseline else cpu_baseline(w, name)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "member-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32+f64", "3xbf16": "f32+bf16x3+f64", "fp32mm": "f32+f64", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": name, "flow": "poiseuille" if w["flow"] else "couette",
                   "Re": w["Re"], "grid": f"{w['Nx']}x{w['Ny']}x{w['Nz']}", "ensemble": E,
                   "dt": w["dt"], "precision": args.precision, "graph": not args.no_graph,
                   "advection": args.advection},
        "grid_point_steps_per_s": value * gp_paper,
        "grid_point_steps_per_s_nominal": value * w["Nx"] * w["Ny"] * w["Nz"],
        "wall_s": wall,
        "kernels": per_kernel,
        "fp64_ms_per_step": fp64["ms_per_step"] if fp64 else None,
        "speedup_vs_fp64": fp64["speedup_of_headline"] if fp64 else None,
        "fp64_step": fp64,
        "serial_gpu_member_steps_per_s": serial,
        "other_advection_form": alternative,
        "tuning": tuning,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
