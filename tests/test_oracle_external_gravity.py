"""Pins of the oracle's uniform external gravity (the free fall g of the
Rayleigh-Taylor test of Sec. 4.4, added to the self-gravity in the Eulerian
stage's sources of Sec. 2).

A uniform state in a periodic box feels only the external field: both
components fall freely, m = rho g t and q = n g t exactly at any step (a
constant force), while the energies approach their closed forms
E = E0 + rho |g|^2 t^2 / 2 and W_ij = W0_ij + n g_i g_j t^2 at first order in
the step (the explicit source uses the momentum at the start of the step)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1311_0861_amd import workloads as W

G_EXT = (0.1, -0.2, 0.05)


def uniform(rho=2.0, nb=0.5, p=1.0, pii=0.3, gamma=5.0 / 3.0):
    one = torch.ones((4, 4, 4), dtype=torch.float64)
    zero = one * 0.0
    Pi = [one * pii, zero, zero, one * pii, zero, one * pii]
    return W.assemble(one * rho, [zero] * 3, one * p, one * nb, [zero] * 3, Pi, gamma)


def falling(steps, dt, g=G_EXT):
    cfg = W.base_config(4, G=0.0, bc=(1, 1, 1), fixed_dt=dt)
    cfg["gext"] = g
    orc = oracle.Oracle(cfg)
    st = uniform()
    orc.set_state(W.to_numpy(st))
    orc.step(steps)
    return orc, W.to_numpy(st)


def test_free_fall_momentum_is_exact():
    T = 0.4
    for n in (8, 16):
        orc, st0 = falling(n, T / n)
        s = orc.get_state()
        for d, comp in enumerate(("x", "y", "z")):
            np.testing.assert_allclose(s["m" + comp], 2.0 * G_EXT[d] * T, rtol=1e-13, atol=1e-15)
            np.testing.assert_allclose(s["q" + comp], 0.5 * G_EXT[d] * T, rtol=1e-13, atol=1e-15)
        for k in ("rho", "n", "Pxy", "Pxz", "Pyz"):  # uniform state: nothing else moves
            np.testing.assert_allclose(s[k], st0[k], rtol=1e-13, atol=1e-15)


def test_free_fall_energies_converge_to_closed_form():
    """E and W approach their closed forms at first order; the internal
    energy and the diagonal stresses, which the energy balance resets to
    E - |m|^2 / 2 rho and W_dd - q_d^2 / n, approach their constant initial
    values at first order too."""
    T = 0.4
    g2 = sum(c * c for c in G_EXT)
    errE, errW, erre, errP = [], [], [], []
    for n in (8, 16, 32):
        orc, st0 = falling(n, T / n)
        s = orc.get_state()
        E_exact = st0["E"] + 0.5 * 2.0 * g2 * T * T
        W_exact = st0["Wxy"] + 0.5 * G_EXT[0] * G_EXT[1] * T * T
        errE.append(float(np.abs(s["E"] - E_exact).max() / np.abs(E_exact).max()))
        errW.append(float(np.abs(s["Wxy"] - W_exact).max() / abs(0.5 * G_EXT[0] * G_EXT[1] * T * T)))
        erre.append(float(np.abs(s["e"] - st0["e"]).max() / np.abs(st0["e"]).max()))
        errP.append(max(float(np.abs(s[k] - st0[k]).max() / np.abs(st0[k]).max()) for k in ("Pxx", "Pyy", "Pzz")))
    for errs in (errE, errW, erre, errP):
        assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.05), errs
        assert errs[1] / errs[2] == pytest.approx(2.0, rel=0.05), errs


def test_no_field_is_the_plain_scheme():
    cfg, st = W.gaussian_blob(8)
    a = oracle.Oracle(cfg)
    b = oracle.Oracle(dict(cfg, gext=(0.0, 0.0, 0.0)))
    for o in (a, b):
        o.set_state(W.to_numpy(st))
        o.step(3)
    sa, sb = a.get_state(), b.get_state()
    assert all(np.array_equal(sa[k], sb[k]) for k in sa)


def test_field_adds_to_self_gravity():
    """With self-gravity on, the external field shifts every cell's momentum
    source by the same rho g tau after one Eulerian stage."""
    cfg, st = W.gaussian_blob(8)
    a = oracle.Oracle(cfg)
    b = oracle.Oracle(dict(cfg, gext=G_EXT))
    for o in (a, b):
        o.set_state(W.to_numpy(st))
        o.stage(0)
    tau = a.diag()[0]["dt"]
    sa, sb = a.get_state(), b.get_state()
    for d, comp in enumerate(("x", "y", "z")):
        np.testing.assert_allclose(sb["m" + comp] - sa["m" + comp], tau * st["rho"].numpy() * G_EXT[d],
                                   rtol=1e-9, atol=1e-15)
        np.testing.assert_allclose(sb["q" + comp] - sa["q" + comp], tau * st["n"].numpy() * G_EXT[d],
                                   rtol=1e-9, atol=1e-15)
