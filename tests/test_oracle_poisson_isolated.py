"""Pins of the oracle's isolated-boundary Poisson solve.

The paper solves Laplace(Phi) = 4 pi G (rho + n) by FFT on a periodic grid
(Sec. 2.3) and cites Hockney and Eastwood's zero-padding method among the
solvers of other codes (Sec. 1).  The isolated form convolves the cell masses
with the sampled point-mass potential -G m / r; the reading for a cell's own
contribution is the potential at the centre of a uniform cube of side h.  The
potential is returned on the grid and on a one-cell ring around it (the
gravity of the outermost cells takes its values there).

Pins, none of them the oracle's own formula:
  - the O(N^6) direct sum of -G m_j / |x_i - x_j| over every source, for
    every output cell of the grid and its ring, on a small non-cubic grid;
    the self term comes from a numerical cube integral here;
  - the analytic free-space potentials of a uniform and a Gaussian sphere
    (no periodic image term, no additive constant), with second-order
    convergence for the smooth one; the Sec. 4.5 sphere rho0 = 1 - r against
    its printed Phi0(r);
  - the discrete self-force sum_i s_i (Phi_{i+1} - Phi_{i-1}) vanishes on
    every axis (the kernel is even), so self-gravity conserves momentum.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def cube_self_integral():
    """Integral of 1/|x| over the unit cube about its centre, numerically."""
    v, _ = integrate.tplquad(lambda z, y, x: 1.0 / math.sqrt(x * x + y * y + z * z), 0, 0.5, 0, 0.5, 0, 0.5,
                             epsabs=1e-13, epsrel=1e-13)
    return 8.0 * v


def direct_sum(s, h, G):
    """Free-space potential of the cell masses at every cell of the grid and
    its one-cell ring, by summing over every source cell."""
    nz, ny, nx = s.shape
    c0 = cube_self_integral()
    out = np.zeros((nz + 2, ny + 2, nx + 2))
    src = [(k, j, i, s[k, j, i]) for k in range(nz) for j in range(ny) for i in range(nx) if s[k, j, i] != 0.0]
    for K in range(-1, nz + 1):
        for J in range(-1, ny + 1):
            for I in range(-1, nx + 1):
                acc = 0.0
                for k, j, i, m in src:
                    r = math.sqrt((I - i) ** 2 + (J - j) ** 2 + (K - k) ** 2)
                    acc += m * (-G * h * h * c0 if r == 0.0 else -G * h * h / r)
                out[K + 1, J + 1, I + 1] = acc
    return out


def test_isolated_equals_direct_sum(orc):
    rng = np.random.default_rng(41)
    s = rng.uniform(0.0, 2.0, size=(4, 6, 8))
    s[1, 2, 3] = 0.0
    h, G = 0.07, 1.3
    got = orc.poisson_isolated(s, h, G)
    ref = direct_sum(s, h, G)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_isolated_single_mass_is_point_potential(orc):
    """One cell of mass m: -G m / r everywhere else, -G m c0 / h at itself,
    whatever the grid (odd offsets, radix-3 lengths)."""
    for shape, pos in (((6, 12, 8), (2, 7, 1)), ((9, 4, 6), (8, 0, 5))):
        s = np.zeros(shape)
        s[pos] = 1.0
        h = 0.1
        phi = orc.poisson_isolated(s, h)
        K, J, I = np.meshgrid(*(np.arange(-1, n + 1) for n in shape), indexing="ij")
        r = np.sqrt((K - pos[0]) ** 2 + (J - pos[1]) ** 2 + (I - pos[2]) ** 2) * h
        m = h ** 3
        ref = np.where(r == 0, -m * cube_self_integral() / h, -m / np.where(r == 0, 1.0, r))
        np.testing.assert_allclose(phi, ref, rtol=1e-11, atol=1e-14)


def _sphere_grid(n, L=1.0):
    h = 2.0 * L / n
    c = -L + (np.arange(-1, n + 1) + 0.5) * h  # grid and its ring
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return h, np.sqrt(X * X + Y * Y + Z * Z)


def test_isolated_gaussian_sphere_converges(orc):
    """Phi = -G M erf(r / (sqrt 2 sigma)) / r, M the grid's mass: the max
    error relative to the central depth falls at second order (measured
    5.8e-3, 2.7e-3, 1.5e-3 at 32, 48, 64 cells)."""
    errs = []
    for n in (32, 48, 64):
        h, r = _sphere_grid(n)
        sig = 0.15
        s = np.exp(-r * r / (2 * sig * sig))[1:-1, 1:-1, 1:-1]
        M = s.sum() * h ** 3
        ref = -M * erf(r / (math.sqrt(2) * sig)) / r
        got = orc.poisson_isolated(s, h)
        errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    assert errs[0] < 8e-3, errs
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.7 * errs[1], errs


def test_isolated_uniform_sphere(orc):
    """Phi = -2 pi G rho0 (R^2 - r^2 / 3) inside, -G M / r outside, with the
    grid's mass M and rho0 = M / (4/3 pi R^3): within 1% of GM/R everywhere
    (the staircase surface), within 0.1% beyond r = 0.5, ring included."""
    n, R = 48, 0.35
    h, r = _sphere_grid(n)
    s = np.where(r <= R, 1.0, 0.0)[1:-1, 1:-1, 1:-1]
    M = s.sum() * h ** 3
    rho0 = M / (4.0 / 3.0 * math.pi * R ** 3)
    ref = np.where(r <= R, -2 * math.pi * rho0 * (R * R - r * r / 3), -M / r)
    err = np.abs(orc.poisson_isolated(s, h) - ref) / (M / R)
    assert err.max() < 1e-2, err.max()
    assert err[r > 0.5].max() < 1e-3, err[r > 0.5].max()


def test_isolated_hydrostatic_sphere_potential(orc):
    """Sec. 4.5: rho0 = 1 - r (r <= 1) on [-2, 2]^3 against the printed
    Phi0(r), inside and out, with no image term and no constant shift."""
    with open(os.path.join(GOLD, "hydrostatic_sphere.json")) as f:
        g = json.load(f)
    assert "pi / (3 r)" in g["phi0_outside"]
    n = 48
    h, r = _sphere_grid(n, L=2.0)
    s = np.where(r <= 1.0, 1.0 - r, 0.0)[1:-1, 1:-1, 1:-1]
    ref = np.where(r <= 1.0, -(math.pi / 3) * (r ** 3 - 2 * r ** 2) - 2 * math.pi / 3, -math.pi / (3 * r))
    err = np.abs(orc.poisson_isolated(s, h) - ref)
    assert err.max() < 2e-2 * (2 * math.pi / 3), err.max()
    assert err[r > 1.2].max() < 2e-3, err[r > 1.2].max()


def test_isolated_self_force_vanishes(orc):
    """sum_i s_i (Phi_{i+e} - Phi_{i-e}) = 0 on each axis: with the central
    difference the grid's own gravity exerts no net force (the kernel is
    even), so isolated self-gravity conserves momentum."""
    rng = np.random.default_rng(7)
    s = rng.uniform(0.0, 1.0, size=(12, 8, 16))
    phi = orc.poisson_isolated(s, 0.1)
    inner = (slice(1, -1),) * 3
    scale = np.abs(s).sum() * np.abs(phi).max()
    for ax in range(3):
        hi = [slice(1, -1)] * 3
        lo = [slice(1, -1)] * 3
        hi[ax] = slice(2, None)
        lo[ax] = slice(0, -2)
        f = (s * (phi[tuple(hi)] - phi[tuple(lo)])).sum()
        assert abs(f) < 1e-14 * scale, (ax, f)
    assert phi[inner].shape == s.shape
