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
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=128, help="cells per axis")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--profile-steps", type=int, default=20, help="steps timed kernel by kernel")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run the library's plain copy kernel over MIB MiB of FP64 data "
                         "(calibrates HBM counters) and exit")
    ap.add_argument("--traffic", default=None,
                    help="JSON with measured HBM bytes per launch of the dominant kernel")
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


def copy_probe(mib):
    """Run the library's device copy kernel (set_field from a device FP64
    tensor into an FP64 sim: reads and writes 8 bytes per cell) 5 times."""
    import torch
    from paper_1311_0861_amd import gpupegas as gp
    from paper_1311_0861_amd import workloads as W
    ncell = mib * 1024 * 1024 // 8
    nz = ncell // (64 * 64)
    cfg = W.base_config((64, 64, nz), lo=(0.0, 0.0, 0.0), hi=(64.0, 64.0, float(nz)), G=0.0)
    sim = gp.Sim(cfg)
    src = torch.ones(nz, 64, 64, dtype=torch.float64, device="cuda")
    for _ in range(5):
        sim.set_field("rho", src)
    sim.sync()
    print(json.dumps({"copy_probe_bytes_read": 8 * 64 * 64 * nz, "copy_probe_bytes_written": 8 * 64 * 64 * nz,
                      "launches": 5}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (one process, one MI355X); "
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
    n = args.n
    cfg_cpu, st_cpu = W.two_disk_collision(n, device="cpu", precision=args.precision)
    ncell = n ** 3

    def fresh_sim():
        s = gp.Sim(cfg_cpu)
        s.set_state({k: v.to("cuda") for k, v in st_cpu.items()})
        return s

    # ---- timed run: warmup, then exactly K graph-replayed steps ------------
    sim = fresh_sim()
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
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        with open(args.traffic) as f:
            tr = json.load(f)
        if tr.get("kernel") == dom and tr.get("n") == n and tr.get("precision") == args.precision:
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": dom,
                "kernel_ms": round(kt[dom], 5), "bytes_per_cell": bpc}
    kernels = {k: {"ms": round(v, 5),
                   "GB/s": round(sim.bytes_per_cell(gp.KERNEL_NAMES.index(k)) * ncell / (v * 1e-3) / 1e9, 1)
                   if v > 0 else None} for k, v in kt.items()}
    step_bytes = sim.bytes_per_cell(-1)
    sim.close()

    # ---- CPU oracle on a bounded sample of the same workload -----------------
    cpu = None
    error = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        orc = oracle.Oracle(cfg_cpu)
        orc.set_state(W.to_numpy(st_cpu))
        orc.dt()  # prologue outside the timed sample
        steps, c0 = 0, time.perf_counter()
        while True:
            orc.step(1)
            steps += 1
            if time.perf_counter() - c0 >= args.cpu_seconds or steps >= 50:
                break
        csec = time.perf_counter() - c0
        cpu = {"value": round(ncell * steps / csec / 1e6, 4), "unit": "Mcell-updates/s",
               "cores": oracle.get_threads(), "kind": "oracle",
               "sample": "%d steps of the same %d^3 two-disk workload from its initial state, FP64, "
                         "plain C + OpenMP" % (steps, n)}
        # the same steps on the GPU from the same inputs give the stated error
        s2 = fresh_sim()
        s2.step(steps)
        s2.sync()
        got = {k: v.cpu().numpy() for k, v in s2.get_state().items()}
        s2.close()
        worst, field = rel_l1_max(got, orc.get_state())
        error = {"vs": "oracle", "metric": "max per-field relative L1", "value": worst, "field": field,
                 "steps": steps}

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
        "step_algorithmic_bytes_per_cell": step_bytes,
        "step_hbm_frac": round(step_bytes * ncell / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
