"""Pins of the oracle's FFT and Poisson solve (Sec. 2.3).

- the FFT equals the direct DFT sum (the definition) and numpy's FFT;
- the potential satisfies the explicit 27-point stencil whose Fourier symbol
  is the one printed in Sec. 2.3 (faces 16, edges 4, corners 1, centre -152,
  over 36 h^2), with the zero mode removed, to round-off;
- an 8^3 dense solve of that stencil gives the same potential;
- a single Fourier mode is scaled exactly by the symbol;
- uniform and Gaussian spheres and the hydrostatic sphere of Sec. 4.5 match
  their analytic potentials (up to the periodic-image background term).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def direct_dft3(x, sign=-1):
    """Direct sum X[k] = sum_m x[m] exp(sign 2 pi i k.m / N), axis by axis."""
    out = x.astype(np.complex128)
    for ax in range(3):
        n = out.shape[ax]
        j = np.arange(n)
        F = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
        out = np.moveaxis(np.tensordot(F, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


def brute_dft3(x):
    """O(N^6) triple sum over all points, for a tiny grid."""
    nz, ny, nx = x.shape
    X = np.zeros_like(x, dtype=np.complex128)
    z, y, w = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for kz, ky, kx in itertools.product(range(nz), range(ny), range(nx)):
        ph = np.exp(-2j * np.pi * (kx * w / nx + ky * y / ny + kz * z / nz))
        X[kz, ky, kx] = np.sum(x * ph)
    return X


@pytest.mark.parametrize("shape", [(4, 6, 8), (9, 12, 2), (27, 1, 16), (18, 24, 6)])
def test_fft_matches_direct_sum(orc, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    got = orc.dft3(x, -1)
    np.testing.assert_allclose(got, direct_dft3(x, -1), rtol=0, atol=1e-11 * np.abs(x).sum())
    np.testing.assert_allclose(got, np.fft.fftn(x), rtol=0, atol=1e-11 * np.abs(x).sum())
    back = orc.dft3(got, +1) / x.size
    np.testing.assert_allclose(back, x, rtol=0, atol=1e-13 * np.abs(x).max() * 10)


def test_fft_brute_force_8cubed(orc):
    rng = np.random.default_rng(8)
    x = rng.normal(size=(8, 8, 8))
    np.testing.assert_allclose(orc.dft3(x, -1), brute_dft3(x), rtol=0, atol=1e-10)


def test_fft_rejects_bad_length(orc):
    with pytest.raises(ValueError):
        orc.dft3(np.zeros((5, 4, 4)), -1)


def stencil27(phi, h):
    """The 27-point operator (16 faces + 4 edges + 1 corners - 152 centre)/(36 h^2)
    with periodic wrap; its symbol is -(6/h^2)(1 - prod_d (1 - 2/3 sin^2))."""
    out = np.zeros_like(phi)
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        nnz = abs(dx) + abs(dy) + abs(dz)
        w = {0: -152.0, 1: 16.0, 2: 4.0, 3: 1.0}[nnz]
        out += w * np.roll(phi, shift=(dz, dy, dx), axis=(0, 1, 2))
    return out / (36.0 * h * h)


@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 16, 6), (24, 18, 32)])
def test_poisson_satisfies_27_point_stencil(orc, shape):
    rng = np.random.default_rng(3)
    s = rng.uniform(0.0, 2.0, size=shape)
    h, G = 0.05, 1.7
    phi = orc.poisson(s, h, G)
    lhs = stencil27(phi, h)
    rhs = 4.0 * math.pi * G * (s - s.mean())
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-11 * np.abs(rhs).max())
    assert abs(phi.mean()) < 1e-13 * np.abs(phi).max()


def test_poisson_printed_sign_would_fail(orc):
    """The symbol as printed (no minus sign) gives -phi; the stencil residual of
    the negated potential is O(1), so the sign reading is pinned."""
    rng = np.random.default_rng(4)
    s = rng.uniform(0.0, 2.0, size=(8, 8, 8))
    phi = orc.poisson(s, 0.1, 1.0)
    rhs = 4.0 * math.pi * (s - s.mean())
    assert np.abs(stencil27(-phi, 0.1) - rhs).max() > 0.5 * np.abs(rhs).max()


def test_poisson_dense_solve_8cubed(orc):
    n, h, G = 8, 0.125, 1.0
    rng = np.random.default_rng(5)
    s = rng.uniform(0.0, 1.0, size=(n, n, n))
    N = n ** 3
    A = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        A[:, c] = stencil27(e.reshape(n, n, n), h).ravel()
    rhs = 4 * math.pi * G * (s - s.mean()).ravel()
    sol = np.linalg.lstsq(A, rhs, rcond=None)[0]
    sol -= sol.mean()
    np.testing.assert_allclose(orc.poisson(s, h, G).ravel(), sol, rtol=0, atol=1e-12 * np.abs(sol).max())


def test_poisson_single_mode(orc):
    nx, ny, nz, h, G = 12, 8, 16, 0.3, 2.0
    kx, ky, kz = 2, 3, 5
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = np.cos(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz))
    D = [1 - 2.0 / 3.0 * math.sin(math.pi * k / m) ** 2 for k, m in ((kx, nx), (ky, ny), (kz, nz))]
    Gk = -4 * math.pi * G * h * h / (6 * (1 - D[0] * D[1] * D[2]))
    np.testing.assert_allclose(orc.poisson(s, h, G), Gk * s, rtol=0, atol=1e-13 * abs(Gk))


def test_poisson_zero_G_and_constant_source(orc):
    s = np.ones((6, 6, 6)) * 3.0
    # only rounding survives: the source minus its mean is zero
    assert np.abs(orc.poisson(s, 0.1, 1.0)).max() < 1e-14 * 4 * math.pi * 3.0
    rng = np.random.default_rng(1)
    assert np.all(orc.poisson(rng.normal(size=(4, 4, 4)), 0.1, 0.0) == 0.0)


def _radial_check(orc, n, L, dens, phi_exact, G=1.0, rmax=0.5):
    h = 2 * L / n
    c = -L + (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    s = dens(r)
    phi = orc.poisson(s, h, G)
    # a periodic solve sees the source minus its mean; the uniform background
    # of density -mean adds -(2 pi / 3) G mean r^2 about the centre (plus the
    # lattice images, which are smooth and small near the centre)
    exact = phi_exact(r) - (2.0 * math.pi / 3.0) * G * s.mean() * r * r
    sel = r <= rmax
    i0 = np.argmin(r)
    got = phi - phi.flat[i0]
    ref = exact - exact.flat[i0]
    return np.abs(got[sel] - ref[sel]).max()


def test_uniform_sphere_potential(orc):
    R, rho0, G = 0.3, 1.0, 1.0
    M = 4.0 / 3.0 * math.pi * R ** 3 * rho0

    def dens(r):
        return np.where(r <= R, rho0, 0.0)

    def pot(r):
        return np.where(r <= R, -2 * math.pi * G * rho0 * (R * R - r * r / 3.0), -G * M / np.maximum(r, 1e-30))

    err = _radial_check(orc, 64, 1.0, dens, pot)
    assert err < 0.01 * G * M / R, err  # the step edge on the grid is O(h)


def test_gaussian_sphere_potential(orc):
    sig, G, M = 0.1, 1.0, 1.0

    def dens(r):
        return M / (2 * math.pi * sig * sig) ** 1.5 * np.exp(-r * r / (2 * sig * sig))

    def pot(r):
        from scipy.special import erf
        rr = np.maximum(r, 1e-12)
        return -G * M * erf(rr / (math.sqrt(2) * sig)) / rr

    err_lo = _radial_check(orc, 32, 1.0, dens, pot)
    err_hi = _radial_check(orc, 64, 1.0, dens, pot)
    scale = G * M / sig
    assert err_hi < 0.01 * scale, err_hi
    assert err_hi < 0.5 * err_lo  # second-order stencil converges


def test_hydrostatic_sphere_potential(orc):
    """rho0 = 1 - r and its closed-form potential Phi0 (Sec. 4.5), G = 1."""
    with open(os.path.join(GOLD, "hydrostatic_sphere.json")) as f:
        ref = json.load(f)
    assert ref["total_mass"] == pytest.approx(math.pi / 3.0, rel=1e-15)

    def dens(r):
        return np.where(r <= 1.0, 1.0 - r, 0.0)

    def pot(r):
        rr = np.maximum(r, 1e-30)
        return np.where(r <= 1.0, -(math.pi / 3.0) * (r ** 3 - 2 * r ** 2) - 2 * math.pi / 3.0,
                        -math.pi / (3.0 * rr))

    err = _radial_check(orc, 64, 2.0, dens, pot, rmax=0.8)
    assert err < 0.02 * math.pi / 3.0, err
