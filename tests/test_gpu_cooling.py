"""Cooling source (Sec. 2, the -q of the gas energy equations, applied in the
Eulerian stage of Sec. 2.1; power-law stand-in for the unavailable tables):
the HIP path against the FP64 oracle on the same seeded inputs (GPU only)."""
import numpy as np
import pytest

from gpu_helpers import assert_close_fields, gpu_state, make_pair, say

pytestmark = pytest.mark.gpu

# about 6% of the central internal energy per step of the 32^3 galaxy; the
# near-vacuum floor (theta < 1e-3) does not cool
COOL = {"cool_lambda": 1.0, "cool_alpha": 0.5, "cool_theta_min": 1e-3}


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


@pytest.mark.parametrize("case", ["blob16", "blob32_isolated"])
def test_cooling_stage_by_stage(gp, W, case):
    say("cooling stage parity", case)
    cfg, st = W.gaussian_blob(16 if case == "blob16" else 32)
    cfg.update(COOL)
    if case.endswith("isolated"):
        cfg["poisson"] = "isolated"
    sim, orc = make_pair(cfg, st)
    for step in range(3):
        sim.stage(gp.GP_STAGE_EUL)
        orc.stage(0)
        assert_close_fields(gpu_state(sim), orc.get_state(), 1e-13, "cooled eulerian step %d" % step, cfg)
        for s_gpu, s_orc in ((gp.GP_STAGE_LAG, 1), (gp.GP_STAGE_POISSON, 2), (gp.GP_STAGE_FINALIZE, 3)):
            sim.stage(s_gpu)
            orc.stage(s_orc)
        assert_close_fields(gpu_state(sim), orc.get_state(), 1e-13, "cooled step %d" % step, cfg)
        dg, do = sim.diag()[-1], orc.diag()[-1]
        for k in ("dt", "e_gas", "mass_gas", "kappa_gas", "n_sync_gas"):
            assert dg[k] == pytest.approx(do[k], rel=1e-11, abs=1e-300), (k, dg[k], do[k])


def test_cooling_blob_100_steps(gp, W):
    """32^3 galaxy with cooling, 100 steps: 1e-9 relative L1.  Cooling takes
    pressure support away, so the collapse runs differently (the gas ends
    with more total energy than without cooling, 0.093 against 0.065)."""
    say("cooled blob 32^3, 100 steps")
    cfg, st = W.gaussian_blob(32)
    cfg.update(COOL)
    sim, orc = make_pair(cfg, st)
    sim.step(100)
    sim.sync()
    orc.step(100)
    assert_close_fields(gpu_state(sim), orc.get_state(), 1e-9, "cooled blob 100 steps", cfg)
    d = sim.diag()
    assert d[-1]["err"] == 0
    base, _ = make_pair(W.gaussian_blob(32)[0], st)
    base.step(100)
    assert d[-1]["e_gas"] > 1.2 * base.diag()[-1]["e_gas"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cooling_two_disk_128(gp, W, precision):
    """The 128^3 two-disk collision with cooling in the benchmark's launch
    configuration (graph replay, tuned launch sizes)."""
    say("cooled two-disk 128^3", precision)
    cfg, st = W.two_disk_collision(128)
    cfg.update(COOL)
    cfg["precision"] = precision
    sim, orc = make_pair(cfg, st)
    sim.step(3)
    sim.sync()
    orc.step(3)
    tol = 1e-11 if precision == "fp64" else 1e-5
    assert_close_fields(gpu_state(sim), orc.get_state(), tol, "cooled two-disk %s" % precision, cfg,
                        slab_tol=None if precision == "fp64" else 1e-3)
    assert sim.diag()[-1]["err"] == 0


def test_batch_mixes_cooled_and_uncooled_runs(gp, W):
    """A cooled member is bitwise equal to itself alone (the same kernel); an
    uncooled member runs the cooling variant with the source switched off and
    matches its run alone to rounding."""
    import torch
    say("batch with cooled and uncooled runs")
    c0, s0 = W.gaussian_blob(16)
    c1 = dict(c0, **COOL)
    b = gp.Batch([c0, c1])
    for r, s in enumerate((s0, s0)):
        b.set_state(r, {k: v.to("cuda") for k, v in s.items()})
    b.step(5)
    b.sync()
    for r, c in enumerate((c0, c1)):
        sim = gp.Sim(c)
        sim.set_state({k: v.to("cuda") for k, v in s0.items()})
        sim.step(5)
        sim.sync()
        a, m = sim.get_state(), b.get_state(r)
        for k in a:
            if r == 1:
                assert torch.equal(a[k], m[k]), (r, k)
            else:
                den = float(a[k].abs().sum()) or 1.0
                assert float((a[k] - m[k]).abs().sum()) / den < 1e-13, (r, k)
        sim.close()
    b.close()


def test_invalid_cooling_configs(gp, W):
    cfg, _ = W.gaussian_blob(8)
    for bad in ({"cool_lambda": -1.0}, {"cool_theta_min": -0.1}, {"cool_lambda": float("nan")},
                {"cool_alpha": float("inf"), "cool_lambda": 1.0}):
        with pytest.raises(gp.GpError) as e:
            gp.Sim(dict(cfg, **bad))
        assert e.value.status == gp.GP_E_INVALID
