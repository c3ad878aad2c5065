"""Seeded synthetic inputs: deterministic, internally consistent, and shaped
like the paper's workloads (CPU only)."""
import math

import numpy as np
import pytest

from paper_1311_0861_amd import workloads as W


def test_same_seed_same_bits():
    a = W.gaussian_blob(16)[1]
    b = W.gaussian_blob(16)[1]
    for f in W.FIELD_NAMES:
        assert np.array_equal(a[f].numpy(), b[f].numpy())
    c = W.gaussian_blob(16, seeds=(5, 6))[1]
    assert not np.array_equal(a["rho"].numpy(), c["rho"].numpy())


def test_state_is_consistent_with_model_relations():
    cfg, st = W.two_disk_collision(32)
    S = {k: v.numpy() for k, v in st.items()}
    g = cfg["gamma"]
    ekin = (S["mx"] ** 2 + S["my"] ** 2 + S["mz"] ** 2) / (2 * S["rho"])
    np.testing.assert_allclose(S["E"], S["e"] + ekin, rtol=1e-14)
    np.testing.assert_allclose((g - 1) * S["e"], 0.1 * S["rho"] ** g, rtol=1e-13)
    for i, a in enumerate("xyz"):
        for j, b in enumerate("xyz"):
            if j < i:
                continue
            key = a + b
            np.testing.assert_allclose(S["W" + key], S["P" + key] + S["q" + a] * S["q" + b] / S["n"],
                                       rtol=1e-13, atol=1e-300)
    # the stars/dark matter carry 0.9 of the disk mass, the gas 0.1
    h3 = (2.0 / 32) ** 3
    assert 8.0 < (S["n"].sum() - 8e-6 / h3 * 0) / S["rho"].sum() < 9.1


def test_disk_masses_and_rotation():
    cfg, st = W.two_disk_collision(64)
    h3 = (2.0 / 64) ** 3
    mtot = (st["rho"].sum() + st["n"].sum()).item() * h3
    M_g = 4 * math.pi * 1.0 * 0.1 ** 2 * 0.02
    floor = 2 * 1e-6 * 8.0
    # two disks plus the floor, within the discretisation of a 1.3-cell-thick disk
    assert abs(mtot - (2 * M_g + floor)) < 0.1 * 2 * M_g
    # bulk velocities +/- 0.25 along x dominate the momentum of each half
    m = st["mx"].numpy() + st["qx"].numpy()
    assert m[:, :, :32].sum() > 0 > m[:, :, 32:].sum()


def test_ensemble_sizes_and_members():
    sizes = W.ensemble_sizes(48)
    assert set(sizes) <= {64, 96, 128} and len(set(sizes)) == 3
    cfg, st = W.ensemble_member(0)
    assert cfg["n"][0] == sizes[0] and cfg["precision"] == "fp32"
    assert st["rho"].shape == (sizes[0],) * 3


def test_shock_tube_layout():
    cfg, st = W.gas_shock_tube(1, n=64, axis=2)
    assert cfg["n"] == (4, 4, 64) and cfg["bc"] == (1, 1, 0) and cfg["G"] == 0.0
    rho = st["rho"].numpy()
    assert rho[0, 0, 0] == 2.0 and rho[-1, 0, 0] == 1.0


@pytest.mark.parametrize("maker", [W.aksenov, W.hydrostatic_sphere])
def test_verification_states_positive(maker):
    cfg, st = maker()
    assert (st["rho"].numpy() > 0).all() and (st["e"].numpy() > 0).all()


def test_kelvin_helmholtz_state():
    """Sec. 4.4: band |y| <= 0.25 of density 2 moving at +0.5 in a density-1
    flow at -0.5, p = 2.5, the y perturbation only near the interfaces."""
    cfg, st = W.kelvin_helmholtz(64)
    assert cfg["bc"] == (1, 1, 1) and cfg["G"] == 0.0 and cfg["gamma"] == 1.4
    X, Y, _ = (a.numpy() for a in W.cell_centres(cfg))
    S = {k: v.numpy() for k, v in st.items()}
    band = np.abs(Y) <= 0.25
    assert np.all(S["rho"][band] == 2.0) and np.all(S["rho"][~band] == 1.0)
    np.testing.assert_allclose(S["mx"] / S["rho"], np.where(band, 0.5, -0.5), rtol=1e-15)
    np.testing.assert_allclose((cfg["gamma"] - 1) * S["e"], 2.5, rtol=1e-14)
    vy = S["my"] / S["rho"]
    assert np.all(vy[np.abs(np.abs(Y) - 0.25) > 0.01] == 0.0) and 0 < vy.max() <= 0.04


def test_rayleigh_taylor_state_is_hydrostatic():
    """Sec. 4.4: heavy fluid (2) over light (1) under g = 0.1 along -y, with
    p = 2.5 - rho g y, i.e. dp/dy = -rho g on each side and p continuous."""
    cfg, st = W.rayleigh_taylor(64)
    g = -cfg["gext"][1]
    assert g == 0.1 and cfg["bc"] == (1, 0, 1)
    _, Y, _ = (a.numpy() for a in W.cell_centres(cfg))
    S = {k: v.numpy() for k, v in st.items()}
    p = (cfg["gamma"] - 1) * S["e"]
    h = 1.0 / 64
    dpdy = np.diff(p[0, :, 0]) / h
    rho_mid = S["rho"][0, :-1, 0]
    same = S["rho"][0, 1:, 0] == rho_mid
    np.testing.assert_allclose(dpdy[same], -rho_mid[same] * g, rtol=1e-9)
    assert np.all(S["rho"][Y <= 0] == 1.0) and np.all(S["rho"][Y > 0] == 2.0)


def test_hydrostatic_sphere_profile_solves_the_equilibrium():
    """The closed forms of Sec. 4.5 satisfy dp/dr = -M(r) rho / r^2 and
    dPhi/dr = M(r) / r^2 with M(r) = 4 pi (r^3 / 3 - r^4 / 4) (G = 1), and
    the potential is continuous at r = 1."""
    import torch
    r = torch.linspace(0.05, 1.5, 300, dtype=torch.float64)
    eps = 1e-6
    rho, p, phi = W.sphere_profile(r)
    _, pp, php = W.sphere_profile(r + eps)
    _, pm, phm = W.sphere_profile(r - eps)
    M = 4 * math.pi * torch.where(r <= 1, r ** 3 / 3 - r ** 4 / 4, torch.full_like(r, 1 / 12.0))
    ok = (r - 1).abs() > 2 * eps
    np.testing.assert_allclose(((pp - pm) / (2 * eps))[ok].numpy(), (-M * rho / r ** 2)[ok].numpy(), atol=1e-7)
    np.testing.assert_allclose(((php - phm) / (2 * eps))[ok].numpy(), (M / r ** 2)[ok].numpy(), rtol=1e-7)
    one = torch.tensor([1.0 - 1e-12, 1.0 + 1e-12], dtype=torch.float64)
    ph = W.sphere_profile(one)[2].numpy()
    assert abs(ph[0] - ph[1]) < 1e-10
    assert 4 * math.pi * (1 / 3 - 1 / 4) == pytest.approx(math.pi / 3)


def test_cloud_collision_state_is_mirror_symmetric():
    cfg, st = W.cloud_collision((48, 32, 32))
    S = {k: v.numpy() for k, v in st.items()}
    assert cfg["poisson"] == "isolated" and cfg["G"] == 1.0
    # to rounding: the cell centres and the order of the two spheres' sums
    np.testing.assert_allclose(S["rho"], S["rho"][:, :, ::-1], rtol=1e-12, atol=0)
    np.testing.assert_allclose(S["mx"], -S["mx"][:, :, ::-1], rtol=1e-12, atol=1e-15)
    h = 4.8 / 48
    mass = (S["rho"].sum() - 1e-3 * S["rho"].size) * h ** 3
    assert mass == pytest.approx(2 * math.pi / 3, rel=0.05)  # two spheres of mass pi / 3
