"""Isolated (zero-padded) Poisson boundaries: the HIP path against the FP64
oracle on the same seeded inputs (GPU only).

The oracle's isolated solve is pinned on the CPU by the O(N^6) direct sum,
the point mass, the analytic spheres and the vanishing self-force
(test_oracle_poisson_isolated.py).  Here the GPU's potential, its one-cell
ring (through the gravity of the outermost cells), the spectral potential
energy and whole steps are compared with it, in both precisions, on even and
radix-3 padded lengths, non-cubic grids and a batch that mixes boundaries.
"""
import math

import numpy as np
import pytest

from gpu_helpers import assert_close_fields, gpu_state, make_pair, say

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


def _iso(cfg, precision="fp64", bc=None):
    c = dict(cfg)
    c["poisson"] = "isolated"
    c["precision"] = precision
    if bc is not None:
        c["bc"] = bc
    return c


def _rel(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum()), float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("shape", [(8, 8, 8), (16, 12, 8), (18, 6, 4), (24, 16, 12), (32, 32, 32)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_isolated_potential_vs_oracle(gp, W, shape, precision):
    """Phi of a random positive density (even, radix-3 and odd half lengths of
    the padded axes, non-cubic grids) and its potential energy."""
    import oracle
    say("isolated potential", shape, precision)
    cfg, st = W.random_periodic(n=shape, seed=11)
    cfg = _iso(cfg, precision, bc=(0, 0, 0))
    sim = gp.Sim(cfg)
    sim.set_state({k: v.to("cuda") for k, v in st.items()})
    got = sim.get_field("phi").cpu().numpy().astype(np.float64)
    s = (st["rho"] + st["n"]).numpy()
    h = (cfg["hi"][0] - cfg["lo"][0]) / cfg["n"][0]
    ref = oracle.poisson_isolated(s, h, cfg["G"])[1:-1, 1:-1, 1:-1]
    l1, mx = _rel(got, ref)
    tol = 1e-12 if precision == "fp64" else 2e-6
    say("  rel L1 %.2e, element-wise %.2e" % (l1, mx))
    assert l1 < tol and mx < 10 * tol, (l1, mx)
    # spectral potential energy (Parseval over the padded lattice) = 1/2 h^3 sum s Phi
    epot = 0.5 * h ** 3 * float((s * ref).sum())
    d = sim.diag()[-1]
    assert d["e_pot"] == pytest.approx(epot, rel=1e-11 if precision == "fp64" else 1e-6)
    sim.close()


@pytest.mark.parametrize("case", ["blob16", "blob32", "disk_24x16x12"])
def test_isolated_stage_by_stage(gp, W, case):
    """Each stage against the oracle; the Eulerian comparison covers the
    outermost cells, whose gravity reads the potential's ring."""
    say("isolated stage parity", case)
    if case == "blob16":
        cfg, st = W.gaussian_blob(16)
    elif case == "blob32":
        cfg, st = W.gaussian_blob(32)
    else:
        cfg, st = W.random_periodic(n=(24, 16, 12), seed=5)
        cfg["bc"] = (0, 0, 0)
    cfg = _iso(cfg)
    sim, orc = make_pair(cfg, st)
    for step in range(2):
        a = sim.get_field("phi").cpu().numpy()
        l1, mx = _rel(a, orc.get_field("phi"))
        assert l1 < 1e-12 and mx < 1e-11, (step, l1, mx)
        sim.stage(gp.GP_STAGE_EUL)
        orc.stage(0)
        assert_close_fields(gpu_state(sim), orc.get_state(), 1e-13, "eulerian step %d" % step, cfg)
        sim.stage(gp.GP_STAGE_LAG)
        orc.stage(1)
        assert_close_fields(gpu_state(sim), orc.get_state(), 1e-13, "lagrangian step %d" % step, cfg)
        sim.stage(gp.GP_STAGE_POISSON)
        orc.stage(2)
        sim.stage(gp.GP_STAGE_FINALIZE)
        orc.stage(3)
        dg, do = sim.diag()[-1], orc.diag()[-1]
        for k in ("t", "dt", "mass_gas", "mass_bme", "e_gas", "e_bme", "e_pot", "kappa_gas", "kappa_bme"):
            assert dg[k] == pytest.approx(do[k], rel=1e-11, abs=1e-300), (k, dg[k], do[k])
        assert dg["step"] == do["step"] and dg["err"] == 0


def test_isolated_blob_100_steps(gp, W):
    """Single Gaussian galaxy, 32^3, isolated potential, 100 steps: 1e-9."""
    say("isolated blob 32^3, 100 steps")
    cfg, st = W.gaussian_blob(32)
    cfg = _iso(cfg)
    sim, orc = make_pair(cfg, st)
    sim.step(100)
    sim.sync()
    orc.step(100)
    assert_close_fields(gpu_state(sim), orc.get_state(), 1e-9, "isolated blob 100 steps", cfg)
    dg, do = sim.diag(), orc.diag()
    assert len(dg) == len(do)
    for a, b in zip(dg, do):
        assert a["e_pot"] == pytest.approx(b["e_pot"], rel=1e-9)
        assert a["dt"] == pytest.approx(b["dt"], rel=1e-9)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_isolated_two_disk_128(gp, W, precision):
    """The two-disk collision at 128^3 with isolated boundaries, in the launch
    configuration the benchmark times (graph replay, tuned launch sizes)."""
    say("isolated two-disk 128^3", precision)
    cfg, st = W.two_disk_collision(128)
    cfg = _iso(cfg, precision)
    sim, orc = make_pair(cfg, st)
    sim.step(3)
    sim.sync()
    orc.step(3)
    tol = 1e-11 if precision == "fp64" else 1e-5
    slab = None if precision == "fp64" else 1e-3
    assert_close_fields(gpu_state(sim), orc.get_state(), tol, "isolated two-disk %s" % precision, cfg,
                        slab_tol=slab)
    a = sim.get_field("phi").cpu().numpy().astype(np.float64)
    l1, mx = _rel(a, orc.get_field("phi"))
    assert l1 < (1e-12 if precision == "fp64" else 1e-6), l1
    d = sim.diag()[-1]
    assert d["err"] == 0
    m0 = sim.diag()[0]
    for comp in ("gas", "bme"):
        drift = abs(d["mass_" + comp] + d["outflow_" + comp] - m0["mass_" + comp]) / m0["mass_" + comp]
        assert drift < 1e-12, (comp, drift)


def test_isolated_uniform_sphere_128(gp, W):
    """A property that holds at any size: the potential of a uniform sphere
    (R = 0.4, total density 1) at 128^3 matches the free-space closed form,
    -2 pi G rho0 (R^2 - r^2 / 3) inside and -G M / r outside, to O(h^2) from
    the cube-sampled surface, with no periodic image term."""
    import torch
    say("isolated uniform sphere 128^3")
    cfg = W.base_config(128, poisson="isolated")
    X, Y, Z = W.cell_centres(cfg, "cuda")
    r = torch.sqrt(X * X + Y * Y + Z * Z)
    R = 0.4
    rho = torch.where(r <= R, torch.ones_like(r), torch.full_like(r, 1e-12))
    zero = torch.zeros_like(r)
    half = 0.5 * rho
    st = W.assemble(half, [zero] * 3, 0.1 * half, half, [zero] * 3,
                    [0.1 * half, zero, zero, 0.1 * half, zero, 0.1 * half], cfg["gamma"])
    sim = gp.Sim(cfg)
    sim.set_state(st)
    phi = sim.get_field("phi").cpu().numpy()
    rr = r.cpu().numpy()
    h = 2.0 / 128
    M = float((rho.cpu().numpy()).sum()) * h ** 3
    exact = np.where(rr <= R, -2.0 * math.pi * (R * R - rr * rr / 3.0), -M / np.maximum(rr, 1e-12))
    band = np.abs(rr - R) > 2 * h  # away from the stair-stepped surface
    err = np.abs(phi - exact)[band].max() / (M / R)
    say("  max error off the surface %.2e of GM/R" % err)
    assert err < 2e-3, err
    sim.close()


def test_batch_mixes_boundaries(gp, W):
    """Runs of one grid size with periodic and isolated potentials (two size
    classes), plus an isolated run of another size, in one batch: every
    member bitwise equal to the same run alone."""
    import torch
    say("batch mixing periodic and isolated potentials")
    c1, s1 = W.gaussian_blob(16)
    c2 = _iso(c1)
    c3, s3 = W.random_periodic(n=(24, 16, 12), seed=4)
    c3 = _iso(c3, bc=(0, 0, 0))
    cfgs, states = [c1, c2, c3, c2], [s1, s1, s3, s1]
    b = gp.Batch(cfgs)
    for r, st in enumerate(states):
        b.set_state(r, {k: v.to("cuda") for k, v in st.items()})
    b.step(6)
    b.sync()
    for r, (c, st) in enumerate(zip(cfgs, states)):
        sim = gp.Sim(c)
        sim.set_state({k: v.to("cuda") for k, v in st.items()})
        sim.step(6)
        sim.sync()
        a, m = sim.get_state(), b.get_state(r)
        for k in a:
            assert torch.equal(a[k], m[k]), (r, k)
        assert torch.equal(sim.get_field("phi"), b.get_field(r, "phi")), r
        assert sim.diag()[-1]["e_pot"] == b.diag(r)[-1]["e_pot"]
        sim.close()
    b.close()
