"""Shared helpers of the GPU parity tests: running the HIP path and the CPU
oracle on the same seeded inputs and comparing field by field."""
import sys

import numpy as np

GROUPS = [["rho"], ["mx", "my", "mz"], ["E"], ["e"], ["n"], ["qx", "qy", "qz"],
          ["Pxx", "Pxy", "Pxz", "Pyy", "Pyz", "Pzz"], ["Wxx", "Wxy", "Wxz", "Wyy", "Wyz", "Wzz"]]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l1(got, ref):
    """Per-field relative L1 error; vector and tensor components are normalised
    by the sum of magnitudes over their whole group, so components that start
    at zero are well defined."""
    out = {}
    for grp in GROUPS:
        den = sum(np.abs(ref[f]).sum() for f in grp)
        for f in grp:
            out[f] = float(np.abs(got[f] - ref[f]).sum() / den) if den > 0 else float(np.abs(got[f]).sum())
    return out


def gpu_state(sim):
    return {k: v.cpu().numpy() for k, v in sim.get_state().items()}


def make_pair(cfg, state):
    """(gpu sim, oracle) set to the same state."""
    import torch
    import oracle
    from paper_1311_0861_amd import gpupegas as gp
    from paper_1311_0861_amd import workloads as W
    sim = gp.Sim(cfg)
    sim.set_state({k: v.to("cuda") for k, v in state.items()})
    orc = oracle.Oracle(cfg)
    orc.set_state(W.to_numpy(state))
    torch.cuda.synchronize()
    return sim, orc


def assert_close_fields(got, ref, tol, what=""):
    err = rel_l1(got, ref)
    worst = max(err, key=err.get)
    assert err[worst] <= tol, "%s: worst field %s rel L1 %.3e > %.1e; all %s" % (
        what, worst, err[worst], tol, {k: "%.1e" % v for k, v in err.items()})
    return err
