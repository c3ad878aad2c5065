"""The oracle on the verification problems of Sec. 4.4 (Kelvin-Helmholtz) and
Sec. 4.5 (two colliding hydrostatic gas clouds): properties that the paper's
setups fix exactly, since it reports them as figures only (CPU)."""
import numpy as np

import oracle
from paper_1311_0861_amd import workloads as W


def test_kelvin_helmholtz_conserves_mass_and_momentum():
    """Periodic on every axis with no gravity: total mass and momentum stay
    at their initial values to rounding while the shear layer evolves."""
    cfg, st = W.kelvin_helmholtz(64)  # at 32^2 no cell centre falls inside the perturbed strips
    orc = oracle.Oracle(cfg)
    orc.set_state(W.to_numpy(st))
    orc.step(40)
    d = orc.diag()
    m0 = d[0]["mass_gas"]
    for r in d:
        assert abs(r["mass_gas"] - m0) / m0 < 1e-14
        assert abs(r["mom_x"] - d[0]["mom_x"]) < 1e-13 * m0
        assert abs(r["mom_y"] - d[0]["mom_y"]) < 1e-13 * m0
    assert d[-1]["err"] == 0
    s = orc.get_state()
    vy = s["my"] / s["rho"]
    vy0 = (st["my"] / st["rho"]).numpy()
    assert np.abs(vy - vy0).max() > 1e-3  # the perturbed layers have evolved


def test_cloud_collision_keeps_its_mirror_symmetry():
    """The two clouds are mirror images in x (isolated potential, outflow
    boundaries): after 8 steps the density stays even and the x momentum odd
    in x, to rounding, and the clouds approach each other."""
    cfg, st = W.cloud_collision((48, 32, 32))
    orc = oracle.Oracle(cfg)
    orc.set_state(W.to_numpy(st))
    orc.step(8)
    s = orc.get_state()
    assert orc.diag()[-1]["err"] == 0
    rho, mx = s["rho"], s["mx"]
    assert np.abs(rho - rho[:, :, ::-1]).max() < 1e-11 * np.abs(rho).max()
    assert np.abs(mx + mx[:, :, ::-1]).max() < 1e-11 * np.abs(mx).max()
    x = W.cell_centres(cfg)[0][0, 0].numpy()
    prof0 = st["rho"].numpy().sum(axis=(0, 1))
    prof = rho.sum(axis=(0, 1))
    left = x < 0
    c0 = (x[left] * prof0[left]).sum() / prof0[left].sum()
    c1 = (x[left] * prof[left]).sum() / prof[left].sum()
    assert c1 > c0  # the left cloud's centre of mass moved right
