"""Benchmark: Mcell-updates/s of the full GPUPEGAS timestep (Eulerian stage,
FlIC Lagrangian stage, FFT Poisson, CFL/diagnostics reductions) on one MI355X.

Default workload: two colliding exponential disks (gas + stars/dark matter),
128^3 cells over [-1, 1]^3, FP64, CFL 0.2, G = 1, outflow boundaries.
Prints one JSON line; see --help.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=128, help="cells per axis")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--profile-steps", type=int, default=20, help="steps timed kernel by kernel")
    ap.add_argument("--error-steps", type=int, default=100,
                    help="steps of the oracle reference run (its all-thread timing is the CPU baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP32 (256^3, 512^3) and 48-run ensemble measurements")
    ap.add_argument("--form-steps", type=int, default=100, help="timed steps of the extra forms")
    ap.add_argument("--only-form", choices=["fp32_512", "isolated_128", "batch48"], default=None,
                    help="run only this extra form and print its record (for profiler runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run the library's plain copy kernel over MIB MiB of FP64 data "
                         "(calibrates HBM counters) and exit")
    ap.add_argument("--traffic", default=None,
                    help="counter summary with the measured HBM bytes per launch of the dominant kernel "
                         "(default: the one under profiles/ for this size and precision)")
    ap.add_argument("--print-source-hash", action="store_true",
                    help="print the hash of the library sources that traffic figures are tied to and exit")
    return ap.parse_args()


def rel_l1_max(got, ref):
    import numpy as np
    groups = [["rho"], ["mx", "my", "mz"], ["E"], ["e"], ["n"], ["qx", "qy", "qz"],
              ["Pxx", "Pxy", "Pxz", "Pyy", "Pyz", "Pzz"], ["Wxx", "Wxy", "Wxz", "Wyy", "Wyz", "Wzz"]]
    worst, where = 0.0, None
    for g in groups:
        den = sum(float(np.abs(ref[f]).sum()) for f in g)
        for f in g:
            e = float(np.abs(got[f] - ref[f]).sum()) / den
            if e > worst:
                worst, where = e, f
    return worst, where


def rel_elem_max(got, ref):
    """Largest element-wise error of any field, over the largest |value| of
    its group (grouped as rel_l1_max)."""
    import numpy as np
    groups = [["rho"], ["mx", "my", "mz"], ["E"], ["e"], ["n"], ["qx", "qy", "qz"],
              ["Pxx", "Pxy", "Pxz", "Pyy", "Pyz", "Pzz"], ["Wxx", "Wxy", "Wxz", "Wyy", "Wyz", "Wzz"]]
    worst, where = 0.0, None
    for g in groups:
        den = max(float(np.abs(ref[f]).max()) for f in g)
        for f in g:
            e = float(np.abs(got[f] - ref[f]).max()) / den
            if e > worst:
                worst, where = e, f
    return worst, where


def copy_probe(mib):
    """Run the library's device copy kernel (set_field from a device FP64
    tensor into an FP64 sim: reads and writes 8 bytes per cell) 5 times."""
    import torch
    from paper_1311_0861_amd import gpupegas as gp
    from paper_1311_0861_amd import workloads as W
    ncell = mib * 1024 * 1024 // 8
    nz = max(1, min(1024, ncell // (1024 * 1024)))
    cfg = W.base_config((1024, 1024, nz), lo=(0.0, 0.0, 0.0), hi=(1024.0, 1024.0, float(nz)), G=0.0)
    sim = gp.Sim(cfg)
    src = torch.ones(nz, 1024, 1024, dtype=torch.float64, device="cuda")
    for _ in range(5):
        sim.set_field("rho", src)
    sim.sync()
    print(json.dumps({"copy_probe_bytes_read": 8 * 1024 * 1024 * nz, "copy_probe_bytes_written": 8 * 1024 * 1024 * nz,
                      "launches": 5}), flush=True)


def library_source_hash():
    """SHA-256 over the library's HIP sources and public header: a recorded
    HBM-traffic figure is reported only for the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1311_0861_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".hpp")))
    files.append(os.path.join(ROOT, "include", "gpupegas.h"))
    for path in files:
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, workload, path=None):
    """HBM bytes per launch of `kernel` on `workload` (e.g. two_disk_128_fp64)
    from the committed counter summary profiles/hbm_traffic_<workload>.md (a
    line 'traffic: <kernel> <workload> <bytes> <source hash>'), or None when
    there is none for this kernel, workload and library source."""
    path = path or os.path.join(ROOT, "profiles", "hbm_traffic_%s.md" % workload)
    if not os.path.exists(path):
        return None
    want = library_source_hash()
    with open(path) as f:
        for line in f:
            parts = line.strip().strip("`").split()
            if len(parts) == 5 and parts[0] == "traffic:" and parts[1] == kernel and parts[2] == workload \
                    and parts[4] == want:
                return int(parts[3])
    return None


def launch_table(obj):
    """The autotuner's pick for each per-cell kernel: tile shape, z-chunk cap
    (planes) and persistent workgroups."""
    from paper_1311_0861_amd import gpupegas as gp
    out = {}
    for k in gp.CELL_KERNELS:
        shape, cap = obj.get_tiling(k)
        out[k] = {"tile": ("64x4", "32x8")[shape], "chunk_cap": cap, "workgroups": obj.get_launch(k)}
    return out


def kernel_table(obj, kt, cells, workload):
    """Per-kernel time, algorithmic GB/s and, where the counter summary for
    this workload and source is committed, the measured HBM bytes per launch
    and the GB/s they make."""
    from paper_1311_0861_amd import gpupegas as gp
    out = {}
    for k, v in kt.items():
        alg = obj.bytes_per_cell(gp.KERNEL_NAMES.index(k)) * cells
        row = {"ms": round(v, 5), "GB/s": round(alg / (v * 1e-3) / 1e9, 1) if v > 0 else None}
        tr = recorded_traffic(k, workload)
        if tr is not None and v > 0:
            row["hbm_bytes"] = tr
            row["hbm_GB/s"] = round(tr / (v * 1e-3) / 1e9, 1)
            row["hbm_over_algorithmic"] = round(tr / alg, 3)
        out[k] = row
    return out


def cpu_info():
    """Host CPU as lscpu states it (model name, logical CPUs, threads per
    core, cores per socket, sockets), for the stated CPU baseline."""
    import subprocess
    keys = {"Model name": "model", "CPU(s)": "logical_cpus", "Thread(s) per core": "threads_per_core",
            "Core(s) per socket": "cores_per_socket", "Socket(s)": "sockets"}
    out = {}
    try:
        text = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in text.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys and keys[k.strip()] not in out:
                out[keys[k.strip()]] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if "model" not in out:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        out["model"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return out


def oracle_baseline(cfg, st, ncell, err_steps):
    """The oracle (plain C + OpenMP, FP64, untuned) on the host cores.

    All threads: the `err_steps`-step reference run of the error figures,
    timed in three equal segments; the rate is the median segment.  One
    thread: three samples of one step each from the initial state; the rate
    is their median.  Returns (baseline record, oracle after err_steps)."""
    import statistics
    import oracle
    from paper_1311_0861_amd import workloads as W
    oracle.build(force=False)
    threads = oracle.get_threads()
    orc = oracle.Oracle(cfg)
    orc.set_state(W.to_numpy(st))
    orc.dt()  # prologue (Phi^0, tau^0) outside the timed samples
    seg = [err_steps // 3, err_steps // 3, err_steps - 2 * (err_steps // 3)]
    rates = []
    for k in seg:
        c0 = time.perf_counter()
        orc.step(k)
        rates.append(ncell * k / (time.perf_counter() - c0) / 1e6)
    oracle.set_threads(1)
    one = oracle.Oracle(cfg)
    one.set_state(W.to_numpy(st))
    one.dt()
    rates1 = []
    for _ in range(3):
        c0 = time.perf_counter()
        one.step(1)
        rates1.append(ncell / (time.perf_counter() - c0) / 1e6)
    one.close()
    oracle.set_threads(threads)
    n = round(ncell ** (1.0 / 3.0))
    base = {"value": round(statistics.median(rates), 4), "unit": "Mcell-updates/s", "cores": threads,
            "kind": "oracle", "statistic": "median of 3",
            "sample": "%d steps of the %d^3 two-disk workload from its initial state (FP64, plain C + OpenMP "
                      "on %d threads), timed as three segments of %s steps" % (err_steps, n, threads, seg),
            "segments": [round(r, 4) for r in rates],
            "single_thread": {"value": round(statistics.median(rates1), 4), "unit": "Mcell-updates/s",
                              "cores": 1, "statistic": "median of 3",
                              "sample": "3 x 1 step of the same workload from its initial state",
                              "samples": [round(r, 4) for r in rates1]},
            "cpu": cpu_info()}
    return base, orc


def warm_clocks(obj, seconds=0.25):
    """The first step (in it the autotuner picks each per-cell kernel's
    launch configuration), then graph-replayed steps for about `seconds`, so
    that the timed steps run at the GPU's working clocks (a pass that waits
    on the host between kernels leaves the GPU idle between them and does
    not bring it there)."""
    obj.step(1)
    obj.sync()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        obj.step(10)
        obj.sync()


def timed_steps(obj, steps, warmup):
    """Warm up, then time exactly `steps` graph-replayed steps of a Sim/Batch."""
    import torch
    warm_clocks(obj)
    obj.step(warmup)
    obj.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obj.step(steps)
    obj.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def mass_drift(diag):
    out = 0.0
    for comp in ("gas", "bme"):
        m0 = diag[0]["mass_" + comp]
        out = max(out, max(abs(r["mass_" + comp] + r["outflow_" + comp] - m0) / m0 for r in diag))
    return out


def precision_forms(args):
    """FP32 two-disk at 256^3 against the FP64 GPU step after 100 steps, and the
    FP32 three-disk 512^3 run with per-kernel bandwidth."""
    import torch
    from paper_1311_0861_amd import gpupegas as gp
    from paper_1311_0861_amd import workloads as W
    out = {}
    cfg, st = W.two_disk_collision(256, device="cuda")
    states = {}
    for prec in ("fp64", "fp32"):
        c = dict(cfg)
        c["precision"] = prec
        s = gp.Sim(c)
        s.set_state(st)
        s.step(100)
        s.sync()
        states[prec] = s.get_state()
        if prec == "fp32":
            drift = mass_drift(s.diag())
            sec = timed_steps(s, args.form_steps, 5)
            kt = s.time_kernels(3)
            out["fp32_256"] = {"workload": "two-disk collision 256^3 FP32 (rho, n FP64)",
                               "value": round(256 ** 3 * args.form_steps / sec / 1e6, 2),
                               "unit": "Mcell-updates/s", "steps": args.form_steps,
                               "mass_drift_100_steps": drift,
                               "kernels": kernel_table(s, kt, 256 ** 3, "two_disk_256_fp32")}
        else:
            sec = timed_steps(s, args.form_steps, 5)
            out["fp64_256"] = {"workload": "two-disk collision 256^3 FP64",
                               "value": round(256 ** 3 * args.form_steps / sec / 1e6, 2),
                               "unit": "Mcell-updates/s", "steps": args.form_steps}
        s.close()
    err = {}
    for grp in (["rho"], ["mx", "my", "mz"], ["E"], ["e"], ["n"], ["qx", "qy", "qz"],
                ["Pxx", "Pxy", "Pxz", "Pyy", "Pyz", "Pzz"], ["Wxx", "Wxy", "Wxz", "Wyy", "Wyz", "Wzz"]):
        den = sum(float(states["fp64"][f].abs().sum()) for f in grp)
        for f in grp:
            err[f] = float((states["fp32"][f] - states["fp64"][f]).abs().sum()) / den
    out["fp32_256"]["rel_l1_vs_fp64_gpu_100_steps"] = {k: float("%.3g" % v) for k, v in err.items()}
    out["fp32_256"]["rel_l1_max"] = max(err.values())
    del states
    torch.cuda.empty_cache()
    return out


def form_512(args):
    """The FP32 three-disk collision at 512^3 with per-kernel bandwidth."""
    import torch
    from paper_1311_0861_amd import gpupegas as gp
    from paper_1311_0861_amd import workloads as W
    cfg, st = W.three_disk_collision(512, device="cuda", precision="fp32")
    s = gp.Sim(cfg)
    s.set_state(st)
    del st
    torch.cuda.empty_cache()
    sec = timed_steps(s, 50, 2)
    kt = s.time_kernels(3)
    n = 512 ** 3
    out = {"workload": "three-disk collision 512^3 FP32 (rho, n FP64), 50 steps",
           "value": round(n * 50 / sec / 1e6, 2), "unit": "Mcell-updates/s",
           "mass_drift": mass_drift(s.diag()),
           "kernels": kernel_table(s, kt, n, "three_disk_512_fp32")}
    s.close()
    torch.cuda.empty_cache()
    return out



def isolated_form(args):
    """The headline workload with isolated (zero-padded) Poisson boundaries:
    two-disk collision 128^3 FP64, the free-space potential each step."""
    import torch
    from paper_1311_0861_amd import gpupegas as gp
    from paper_1311_0861_amd import workloads as W
    cfg, st = W.two_disk_collision(128, device="cuda")
    cfg["poisson"] = "isolated"
    s = gp.Sim(cfg)
    s.set_state(st)
    del st
    sec = timed_steps(s, args.form_steps, 5)
    kt = s.time_kernels(3)
    n = 128 ** 3
    fft = sum(kt[k] for k in ("fft_xy_fwd", "fft_z_green", "fft_xy_inv"))
    out = {"workload": "two-disk collision 128^3 FP64, isolated Poisson boundaries (zero padding to 256^3)",
           "value": round(n * args.form_steps / sec / 1e6, 2), "unit": "Mcell-updates/s",
           "steps": args.form_steps, "ms_per_step": round(sec / args.form_steps * 1e3, 5),
           "poisson_ms": round(fft, 5), "mass_drift": mass_drift(s.diag()),
           "kernels": kernel_table(s, kt, n, "two_disk_128_fp64_isolated")}
    s.close()
    torch.cuda.empty_cache()
    return out


def batch_form(args):
    """48 independent two-disk runs (64^3 / 96^3 / 128^3, FP32) advanced together."""
    import torch
    from paper_1311_0861_amd import gpupegas as gp
    from paper_1311_0861_amd import workloads as W
    members = [W.ensemble_member(r, device="cuda") for r in range(48)]
    b = gp.Batch([c for c, _ in members])
    for r, (_, st) in enumerate(members):
        b.set_state(r, st)
    del members
    torch.cuda.empty_cache()
    cells = b.cells()
    sec = timed_steps(b, args.form_steps, 5)
    kt = b.time_kernels(3)
    out = {"workload": "48 two-disk runs, sizes drawn from 64^3/96^3/128^3, FP32, one launch per stage",
           "cells": cells, "value": round(cells * args.form_steps / sec / 1e6, 2), "unit": "Mcell-updates/s",
           "steps": args.form_steps,
           "launch": launch_table(b),
           "kernels": kernel_table(b, kt, cells, "ensemble48_fp32")}
    b.close()
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.print_source_hash:
        print(library_source_hash())
        return
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (one process, one MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1311_0861_amd import gpupegas as gp
    from paper_1311_0861_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.only_form:
        fn = {"fp32_512": form_512, "isolated_128": isolated_form, "batch48": batch_form}[args.only_form]
        print(json.dumps({"form": args.only_form, **fn(args)}), flush=True)
        return
    n = args.n
    cfg_cpu, st_cpu = W.two_disk_collision(n, device="cpu", precision=args.precision)
    ncell = n ** 3

    def fresh_sim():
        s = gp.Sim(cfg_cpu)
        s.set_state({k: v.to("cuda") for k, v in st_cpu.items()})
        return s

    sim = fresh_sim()
    # the tuning step, then steps until the GPU runs at its working clocks
    warm_clocks(sim)

    # ---- timed run: warmup, then exactly K graph-replayed steps ------------
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = t1 - t0
    ms_per_step = sec / args.steps * 1e3
    value = ncell * args.steps / sec / 1e6
    diag = sim.diag()[-1]

    # ---- per-kernel durations with HIP events on the sim's stream -------------
    kt = sim.time_kernels(args.profile_steps)
    dom = max(kt, key=kt.get)
    kid = gp.KERNEL_NAMES.index(dom)
    bpc = sim.bytes_per_cell(kid)
    achieved = bpc * ncell / (kt[dom] * 1e-3) / 1e9
    workload = "two_disk_%d_%s" % (n, args.precision)
    traffic = recorded_traffic(dom, workload, args.traffic)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": dom,
                "kernel_ms": round(kt[dom], 5), "bytes_per_cell": bpc}
    kernels = kernel_table(sim, kt, ncell, workload)
    step_bytes = sim.bytes_per_cell(-1)
    launch = launch_table(sim)
    sim.close()

    # ---- CPU oracle: reference run of the error figures, and the baseline -----
    cpu = None
    error = None
    if not args.no_cpu_baseline:
        cpu, orc = oracle_baseline(cfg_cpu, st_cpu, ncell, args.error_steps)
        ref = orc.get_state()
        error = {"vs": "oracle", "metric": "max per-field relative L1 (and element-wise max error over the "
                                          "group's largest value)", "steps": args.error_steps}
        # the same steps on the GPU from the same inputs, in both precisions
        for prec in ("fp64", "fp32"):
            s2 = gp.Sim(dict(cfg_cpu, precision=prec))
            s2.set_state({k: v.to("cuda") for k, v in st_cpu.items()})
            s2.step(args.error_steps)
            s2.sync()
            got = {k: v.cpu().numpy() for k, v in s2.get_state().items()}
            s2.close()
            worst, field = rel_l1_max(got, ref)
            wmax, fmax = rel_elem_max(got, ref)
            error[prec] = {"value": worst, "field": field, "elementwise": wmax, "elementwise_field": fmax}
        error["value"] = error[args.precision]["value"]
        error["field"] = error[args.precision]["field"]

    forms = None
    if not args.no_forms:
        forms = precision_forms(args)
        forms["fp32_512"] = form_512(args)
        forms["isolated_128"] = isolated_form(args)
        forms["batch48"] = batch_form(args)

    out = {
        "metric": "Mcell-updates/s per full timestep incl. FFT Poisson",
        "value": round(value, 3),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "two-disk galaxy collision (gas + stars/DM), %d^3 over [-1,1]^3, %s, "
                               "CFL 0.2, G=1, outflow" % (n, args.precision.upper()),
                   "cells": ncell, "precision": args.precision, "t_end_of_run": diag["t"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error": error,
        "kernels": kernels,
        "launch": launch,
        "forms": forms,
        "step_algorithmic_bytes_per_cell": step_bytes,
        "step_hbm_frac": round(step_bytes * ncell / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
