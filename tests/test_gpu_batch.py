"""Ensemble (batching) form against standalone runs (GPU only).

A batch advances independent runs of uneven grid sizes together (persistent
per-stage launches over a (run, tile) work list, one FFT launch per grid size,
graph-replayed steps).  Each member must equal the same run in its own sim
bitwise, whatever persistent grid sizes and tilings are used; where whole
diagnostics records are compared bitwise, both sides run the same tiling."""
import numpy as np
import pytest

from gpu_helpers import FP32_SLAB_TOL, assert_close_fields, gpu_state, pin_tiling, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_1311_0861_amd import gpupegas
    return gpupegas


@pytest.fixture(scope="module")
def W():
    from paper_1311_0861_amd import workloads
    return workloads


def _members(W, prec="fp64"):
    out = [W.gaussian_blob(16), W.random_periodic(n=(16, 12, 8), seed=7),
           W.gaussian_blob(16, seeds=(11, 12)), W.gaussian_blob(32),
           W.gas_shock_tube(2, n=64, axis=1)]
    for cfg, _ in out:
        cfg["precision"] = prec
    return out


def _batch_state(b, r):
    return {k: v.cpu().numpy() for k, v in b.get_state(r).items()}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_members_equal_standalone_runs(gp, W, prec):
    say("batch vs standalone", prec)
    members = _members(W, prec)
    b = gp.Batch([c for c, _ in members])
    for r, (_, st) in enumerate(members):
        b.set_state(r, {k: v.to("cuda") for k, v in st.items()})
    b.step(12)
    b.sync()
    for r, (cfg, st) in enumerate(members):
        s = gp.Sim(cfg)
        s.set_state({k: v.to("cuda") for k, v in st.items()})
        s.step(12)
        ref = gpu_state(s)
        got = _batch_state(b, r)
        for f in ref:
            np.testing.assert_array_equal(got[f], ref[f], err_msg="run %d field %s" % (r, f))
        dg, ds = b.diag(r)[-1], s.diag()[-1]
        assert dg["t"] == ds["t"] and dg["e_pot"] == ds["e_pot"] and dg["step"] == 12
        s.close()


def test_batch_result_independent_of_launch_size(gp, W):
    """Persistent grids of 1, 3 and 7 workgroups (fewer than the 8 XCDs, so
    some XCDs get no workgroup), 8, 13 and 24, and one workgroup per item,
    all give the same bits."""
    say("launch size independence")
    members = _members(W)
    runs = []
    sizes = (0, 1, 3, 7, 8, 13, 24)
    for blocks in sizes:
        b = gp.Batch([c for c, _ in members])
        for r, (_, st) in enumerate(members):
            b.set_state(r, {k: v.to("cuda") for k, v in st.items()})
        for k in gp.CELL_KERNELS:
            b.set_launch(k, blocks)
        for k in gp.CELL_KERNELS:
            assert b.get_launch(k) == blocks or blocks == 0
        b.step(5)
        runs.append([_batch_state(b, r) for r in range(len(members))])
        b.close()
    for q in range(1, len(sizes)):
        for r in range(len(members)):
            for f in runs[0][r]:
                np.testing.assert_array_equal(runs[q][r][f], runs[0][r][f],
                                              err_msg="blocks %d run %d field %s" % (sizes[q], r, f))


def test_ensemble_members_radix3(gp, W):
    """Members of the 48-run ensemble drawn so that all three grid sizes
    (64, 96 with its radix-3 FFT, 128) appear, FP32, 4 steps."""
    say("ensemble members with 64/96/128")
    sizes = W.ensemble_sizes(48)
    pick = []
    for n in (64, 96, 128):
        pick.append(sizes.index(n))
    members = [W.ensemble_member(r) for r in pick]
    b = gp.Batch([c for c, _ in members])
    for r, (_, st) in enumerate(members):
        b.set_state(r, {k: v.to("cuda") for k, v in st.items()})
    b.step(4)
    b.sync()
    for r, (cfg, st) in enumerate(members):
        s = gp.Sim(cfg)
        s.set_state({k: v.to("cuda") for k, v in st.items()})
        s.step(4)
        ref = gpu_state(s)
        got = _batch_state(b, r)
        for f in ref:
            np.testing.assert_array_equal(got[f], ref[f], err_msg="member %d field %s" % (pick[r], f))
        s.close()


def test_ensemble_members_against_oracle(gp, W):
    """Three members of the 48-run ensemble (64^3, 96^3 with its radix-3 FFT,
    128^3), FP32, advanced together as one batch in the benchmark's launch
    configuration, each against the FP64 oracle after 4 steps: within 1e-5
    relative L1 per field (FP32 rounding over a few steps), element-wise,
    and on the near-vacuum outflow planes within the FP32 bar of those planes
    (gpu_helpers.FP32_SLAB_TOL); potential and time as well."""
    import oracle
    say("ensemble members 64/96/128 FP32 batched vs the oracle, 4 steps")
    sizes = W.ensemble_sizes(48)
    pick = [sizes.index(n) for n in (64, 96, 128)]
    members = [W.ensemble_member(r) for r in pick]
    b = gp.Batch([c for c, _ in members])
    for r, (_, st) in enumerate(members):
        b.set_state(r, {k: v.to("cuda") for k, v in st.items()})
    b.step(4)
    b.sync()
    for r, (cfg, st) in enumerate(members):
        orc = oracle.Oracle(cfg)
        orc.set_state(W.to_numpy(st))
        orc.step(4)
        assert_close_fields(_batch_state(b, r), orc.get_state(), 1e-5, "member %d (%d^3)" % (pick[r], cfg["n"][0]),
                            cfg, slab_tol=FP32_SLAB_TOL)
        phi = b.get_potential(r).cpu().numpy()
        ref = orc.get_field("phi")
        assert np.abs(phi - ref).sum() / np.abs(ref).sum() < 1e-5
        dg, do = b.diag(r)[-1], orc.diag()[-1]
        assert dg["step"] == 4 and dg["err"] == 0
        assert dg["t"] == pytest.approx(do["t"], rel=1e-5)
        orc.close()
    b.close()


def test_same_size_runs_keep_their_potential_energy(gp, W):
    """Two runs of one grid size whose ny (12) is not a multiple of the z
    pass's 8-line XCD groups, so one group spans both runs: every diagnostics
    record of each member (its potential energy among them) equals that of the
    same run alone, bitwise."""
    say("same-size runs, ny = 12")
    members = [W.random_periodic(n=(16, 12, 8), seed=s) for s in (21, 22)]
    b = gp.Batch([c for c, _ in members])
    pin_tiling(b)
    for r, (_, st) in enumerate(members):
        b.set_state(r, {k: v.to("cuda") for k, v in st.items()})
    b.step(3)
    b.sync()
    for r, (cfg, st) in enumerate(members):
        s = gp.Sim(cfg)
        pin_tiling(s)
        s.set_state({k: v.to("cuda") for k, v in st.items()})
        s.step(3)
        s.sync()
        assert b.diag(r) == s.diag(), r
        ref = gpu_state(s)
        got = _batch_state(b, r)
        for f in ref:
            np.testing.assert_array_equal(got[f], ref[f], err_msg="run %d field %s" % (r, f))
        s.close()
    b.close()


def test_batch_mixing_fft_forms(gp, W):
    """A batch whose size classes take different forms of the Poisson solve: a
    256 x 256 x 4 FP32 run (its half planes do not fit two to a CU, so it takes
    the separate x and y passes) beside a 16 x 12 x 8 one (half planes), with
    the reduction and finalize workgroups riding along in whichever passes come
    first.  Each member equals the same run alone, bitwise."""
    say("batch mixing FFT forms")
    members = [W.random_periodic(n=(256, 256, 4), seed=31), W.random_periodic(n=(16, 12, 8), seed=32)]
    for cfg, _ in members:
        cfg["precision"] = "fp32"
    b = gp.Batch([c for c, _ in members])
    pin_tiling(b)
    for r, (_, st) in enumerate(members):
        b.set_state(r, {k: v.to("cuda") for k, v in st.items()})
    b.step(3)
    b.sync()
    for r, (cfg, st) in enumerate(members):
        s = gp.Sim(cfg)
        pin_tiling(s)
        s.set_state({k: v.to("cuda") for k, v in st.items()})
        s.step(3)
        s.sync()
        assert b.diag(r) == s.diag(), r
        ref = gpu_state(s)
        got = _batch_state(b, r)
        for f in ref:
            np.testing.assert_array_equal(got[f], ref[f], err_msg="run %d field %s" % (r, f))
        s.close()
    b.close()
