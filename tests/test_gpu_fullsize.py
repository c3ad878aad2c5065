"""The precision and batching forms at their full benchmark sizes, in the
launch configuration the benchmark times (graph replay, tuned launch sizes):

- two-disk collision 256^3, FP32 state (the x and y transforms as separate
  passes, since a 256 x 129 plane does not fit in LDS): against the FP64
  oracle and the FP64 GPU step, in full, after 3 steps;
- three-disk collision 512^3, FP32: properties that hold at any size (mass
  balance to 1e-12, no latched errors) and the FP64 GPU step as reference,
  compared on the device;
- the 48-run ensemble (64^3 / 96^3 / 128^3, FP32): every member's mass balance
  and error word, and its largest member bitwise equal to the same run alone.
"""
import numpy as np
import pytest

from gpu_helpers import FP32_SLAB_TOL, assert_close_fields, gpu_state, rel_l1, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1311_0861_amd import gpupegas
    return gpupegas


@pytest.fixture(scope="module")
def W():
    from paper_1311_0861_amd import workloads
    return workloads


def _mass_drift(diag):
    d0 = diag[0]
    return max(abs(r["mass_" + c] + r["outflow_" + c] - d0["mass_" + c]) / d0["mass_" + c]
               for r in diag for c in ("gas", "bme"))


def _device_rel_l1(a, b):
    """Per-field relative L1 of two device states, grouped as in rel_l1."""
    from gpu_helpers import GROUPS
    out = {}
    for grp in GROUPS:
        den = sum(float(b[f].double().abs().sum()) for f in grp)
        for f in grp:
            out[f] = float((a[f].double() - b[f].double()).abs().sum()) / den
    return out


def _run(gp, cfg, st, steps, precision):
    c = dict(cfg)
    c["precision"] = precision
    sim = gp.Sim(c)
    sim.set_state({k: v.to("cuda") for k, v in st.items()})
    sim.step(steps)
    sim.sync()
    return sim


def test_fp32_two_disk_256(gp, W):
    import oracle
    import torch
    say("full size: two-disk 256^3 FP32, 3 steps, against the oracle and the FP64 GPU step")
    cfg, st = W.two_disk_collision(256)
    s32 = _run(gp, cfg, st, 3, "fp32")
    g32 = gpu_state(s32)
    d32 = s32.diag()
    s32.close()
    s64 = _run(gp, cfg, st, 3, "fp64")
    g64 = gpu_state(s64)
    s64.close()
    torch.cuda.empty_cache()
    orc = oracle.Oracle(cfg)
    orc.set_state(W.to_numpy(st))
    orc.step(3)
    ref = orc.get_state()
    assert_close_fields(g64, ref, 1e-12, "FP64 GPU vs oracle, 256^3", cfg)
    assert_close_fields(g32, ref, 1e-5, "FP32 GPU vs oracle, 256^3", cfg, slab_tol=FP32_SLAB_TOL)
    assert max(rel_l1(g32, g64).values()) <= 1e-5
    assert _mass_drift(d32) <= 1e-12
    assert d32[-1]["err"] == 0 and d32[-1]["step"] == 3


def test_fp32_three_disk_512(gp, W):
    import torch
    say("full size: three-disk 512^3 FP32, 2 steps, against the FP64 GPU step")
    cfg, st = W.three_disk_collision(512, device="cuda")
    s32 = _run(gp, cfg, st, 2, "fp32")
    d32 = s32.diag()
    s64 = _run(gp, cfg, st, 2, "fp64")
    del st
    torch.cuda.empty_cache()
    err = _device_rel_l1(s32.get_state(), s64.get_state())
    say("worst FP32 vs FP64 %.2e (%s)" % (max(err.values()), max(err, key=err.get)))
    assert max(err.values()) <= 1e-5, err
    assert _mass_drift(d32) <= 1e-12
    assert d32[-1]["err"] == 0 and s64.diag()[-1]["err"] == 0
    s32.close()
    s64.close()
    torch.cuda.empty_cache()


def test_ensemble_48(gp, W):
    import torch
    say("full size: 48-run ensemble, 3 steps")
    members = [W.ensemble_member(r, device="cuda") for r in range(48)]
    b = gp.Batch([c for c, _ in members])
    for r, (_, st) in enumerate(members):
        b.set_state(r, st)
    b.step(3)
    b.sync()
    for r in range(48):
        d = b.diag(r)
        assert d[-1]["err"] == 0 and d[-1]["step"] == 3, r
        assert _mass_drift(d) <= 1e-12, r
    big = max(range(48), key=lambda r: members[r][0]["n"][0])
    cfg, st = members[big]
    alone = gp.Sim(cfg)
    alone.set_state(st)
    alone.step(3)
    alone.sync()
    got, ref = b.get_state(big), alone.get_state()
    for k in gp.FIELD_NAMES:
        assert torch.equal(got[k], ref[k]), (big, k)
    assert np.array_equal(b.get_field(big, "phi").cpu().numpy(), alone.get_field("phi").cpu().numpy())
    alone.close()
    b.close()
    del members
    torch.cuda.empty_cache()
