"""Seeded synthetic initial states for the GPUPEGAS timestep.

This module holds no arithmetic of the numerical method: it only builds
initial fields from closed-form profiles and seeded noise.  It is the one
module that both the GPU path's callers and the CPU oracle's tests use, so
that both sides start from the same bits.

All arrays are float64 tensors shaped (nz, ny, nx), x fastest.  Fields follow
the state order of the library: gas (rho, rho v, rho E, rho eps) and the
Boltzmann-moment component (n, n u, Pi_ij, n E_ij = Pi_ij + n u_i u_j), with
rho E = rho eps + rho v^2 / 2 and p = (gamma - 1) rho eps (Sec. 2 of the paper).

Noise is drawn with numpy's PCG64 in C order of shape (nz, ny, nx), so the
same seed gives the same field whatever the device the profile is built on.
"""
import math

import numpy as np
import torch

FIELD_NAMES = [
    "rho", "mx", "my", "mz", "E", "e",
    "n", "qx", "qy", "qz",
    "Pxx", "Pxy", "Pxz", "Pyy", "Pyz", "Pzz",
    "Wxx", "Wxy", "Wxz", "Wyy", "Wyz", "Wzz",
]
_SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]

DEFAULT_GAMMA = 5.0 / 3.0


def base_config(n, lo=-1.0, hi=1.0, gamma=DEFAULT_GAMMA, G=1.0, cfl=0.2,
                eta=1e-3, bc=(0, 0, 0), fixed_dt=0.0, t_end=0.0, precision="fp64", poisson="periodic"):
    """Run configuration as a plain dict (both the library and the oracle read
    it).  poisson: "periodic" or "isolated" boundaries of the potential."""
    if isinstance(n, int):
        n = (n, n, n)
    lo = tuple(lo) if isinstance(lo, (tuple, list)) else (lo,) * 3
    hi = tuple(hi) if isinstance(hi, (tuple, list)) else (hi,) * 3
    return dict(n=tuple(int(v) for v in n), lo=lo, hi=hi, gamma=gamma, G=G,
                cfl=cfl, eta=eta, bc=tuple(bc), fixed_dt=fixed_dt, t_end=t_end,
                precision=precision, poisson=poisson)


def cell_centres(cfg, device="cpu"):
    """Cell-centre coordinates lo + (i + 1/2) h as three (nz, ny, nx) tensors."""
    nx, ny, nz = cfg["n"]
    ax = []
    for d, nd in enumerate((nx, ny, nz)):
        h = (cfg["hi"][d] - cfg["lo"][d]) / nd
        ax.append(cfg["lo"][d] + (torch.arange(nd, dtype=torch.float64, device=device) + 0.5) * h)
    Z, Y, X = torch.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def normal_noise(seed, shape, device="cpu"):
    """Standard normal noise from PCG64(seed), drawn in C order of `shape`."""
    g = np.random.Generator(np.random.PCG64(seed))
    return torch.from_numpy(g.standard_normal(size=shape)).to(device)


def assemble(rho, v, p, n, u, Pi, gamma):
    """Conserved state from primitive fields.  v, u: lists of 3 tensors;
    Pi: list of 6 tensors in slot order xx, xy, xz, yy, yz, zz."""
    e = p / (gamma - 1.0)
    st = {"rho": rho, "mx": rho * v[0], "my": rho * v[1], "mz": rho * v[2],
          "E": e + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2), "e": e,
          "n": n, "qx": n * u[0], "qy": n * u[1], "qz": n * u[2]}
    for s, (i, j) in enumerate(_SYM):
        st["P" + "xyz"[i] + "xyz"[j]] = Pi[s]
        st["W" + "xyz"[i] + "xyz"[j]] = Pi[s] + n * u[i] * u[j]
    return {k: st[k].contiguous() for k in FIELD_NAMES}


# --------------------------------------------------------------------------
# Single Gaussian galaxy (32^3, FP64, 100 steps)

def gaussian_blob(n=32, device="cpu", seeds=(1, 2), sigma=0.2, noise=0.01):
    cfg = base_config(n)
    X, Y, Z = cell_centres(cfg, device)
    r2 = X * X + Y * Y + Z * Z
    prof = torch.exp(-r2 / (2.0 * sigma * sigma)) + 1e-6
    shape = tuple(X.shape)
    rho = prof * (1.0 + noise * normal_noise(seeds[0], shape, device))
    nb = prof * (1.0 + noise * normal_noise(seeds[1], shape, device))
    g = cfg["gamma"]
    zero = torch.zeros_like(rho)
    p = 0.1 * rho ** g
    pii = 0.05 * nb ** g
    Pi = [pii, zero, zero, pii.clone(), zero, pii.clone()]
    return cfg, assemble(rho, [zero] * 3, p, nb, [zero] * 3, Pi, g)


# --------------------------------------------------------------------------
# Colliding exponential disks

def rot_y(theta):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_axis(axis, theta):
    """Rotation by theta about a unit axis (Rodrigues)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(theta) * K + (1 - math.cos(theta)) * (K @ K)


def disk_collision(n, galaxies, noise_seeds, device="cpu", rho_c=1.0, R_d=0.1,
                   z_0=0.02, gas_frac=0.1, G=1.0, precision="fp64"):
    """Exponential disks rho_c exp(-R/R_d) sech^2(z/z_0) with a circular velocity
    from the enclosed mass M(<R) = M_g [1 - (1 + R/R_d) exp(-R/R_d)].
    galaxies: list of dicts with centre c (3), bulk velocity V (3), rotation R
    (3x3, disk frame -> lab)."""
    cfg = base_config(n, precision=precision, G=G)
    g = cfg["gamma"]
    X, Y, Z = cell_centres(cfg, device)
    M_g = 4.0 * math.pi * rho_c * R_d * R_d * z_0
    tot = torch.zeros_like(X)
    mom = [torch.zeros_like(X) for _ in range(3)]
    for gal in galaxies:
        c = gal["c"]
        Rm = torch.as_tensor(np.asarray(gal["R"], dtype=np.float64), device=device)
        dx = [X - c[0], Y - c[1], Z - c[2]]
        # disk-frame coordinates y = R^T (x - c)
        yv = [Rm[0, k] * dx[0] + Rm[1, k] * dx[1] + Rm[2, k] * dx[2] for k in range(3)]
        R = torch.sqrt(yv[0] ** 2 + yv[1] ** 2)
        rg = rho_c * torch.exp(-R / R_d) / torch.cosh(yv[2] / z_0) ** 2
        Rs = torch.clamp(R, min=1e-12)
        xr = Rs / R_d
        menc = M_g * (1.0 - (1.0 + xr) * torch.exp(-xr))
        vrot = torch.sqrt(G * menc / Rs)
        tdir = [-yv[1] / Rs, yv[0] / Rs, torch.zeros_like(Rs)]  # disk frame
        for k in range(3):
            lab_t = Rm[k, 0] * tdir[0] + Rm[k, 1] * tdir[1] + Rm[k, 2] * tdir[2]
            mom[k] = mom[k] + rg * (gal["V"][k] + vrot * lab_t)
        tot = tot + rg
    vel = [m / (tot + 1e-6) for m in mom]
    shape = tuple(X.shape)
    rho = (gas_frac * tot + 1e-6) * torch.exp(0.01 * normal_noise(noise_seeds[0], shape, device) - 0.5e-4)
    nb = ((1.0 - gas_frac) * tot + 1e-6) * torch.exp(0.01 * normal_noise(noise_seeds[1], shape, device) - 0.5e-4)
    p = 0.1 * rho ** g
    pii = 0.05 * nb ** g
    zero = torch.zeros_like(rho)
    Pi = [pii, zero, zero, pii.clone(), zero, pii.clone()]
    return cfg, assemble(rho, vel, p, nb, vel, Pi, g)


def two_disk_collision(n=128, device="cpu", precision="fp64"):
    """Head-on pair: centres x = -/+0.3, velocities +/-0.25, second disk tilted
    30 degrees about y; noise seeds 3 (gas) and 4 (stars/dark matter)."""
    gals = [dict(c=(-0.3, 0.0, 0.0), V=(0.25, 0.0, 0.0), R=np.eye(3)),
            dict(c=(0.3, 0.0, 0.0), V=(-0.25, 0.0, 0.0), R=rot_y(math.radians(30.0)))]
    return disk_collision(n, gals, (3, 4), device, precision=precision)


def three_disk_collision(n=512, device="cpu", precision="fp32", seed=5):
    """Three disks at seeded positions |c| < 0.5, velocities |V| < 0.5 and tilts
    U(0, 90 deg) about a random in-plane axis; noise seeds 6 and 7."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def in_ball(radius):
        while True:
            p = rng.uniform(-radius, radius, 3)
            if np.linalg.norm(p) < radius:
                return p

    gals = []
    for _ in range(3):
        c = in_ball(0.5)
        V = in_ball(0.5)
        theta = math.radians(rng.uniform(0.0, 90.0))
        phi = rng.uniform(0.0, 2.0 * math.pi)
        gals.append(dict(c=tuple(c), V=tuple(V), R=rot_axis((math.cos(phi), math.sin(phi), 0.0), theta)))
    return disk_collision(n, gals, (6, 7), device, precision=precision)


def ensemble_member(r, device="cpu", precision="fp32", base_seed=1311):
    """Member r of the 48-run ensemble: N in {64, 96, 128}, impact parameter
    b ~ U(0, 0.4), relative speed U(0.2, 0.8), tilt of disk 2 U(0, 90 deg)."""
    rng = np.random.Generator(np.random.PCG64([base_seed, r]))
    n = int(rng.choice([64, 96, 128]))
    b = rng.uniform(0.0, 0.4)
    vrel = rng.uniform(0.2, 0.8)
    theta = math.radians(rng.uniform(0.0, 90.0))
    gals = [dict(c=(-0.3, -b / 2, 0.0), V=(vrel / 2, 0.0, 0.0), R=np.eye(3)),
            dict(c=(0.3, b / 2, 0.0), V=(-vrel / 2, 0.0, 0.0), R=rot_y(theta))]
    seeds = ([base_seed, r, 0], [base_seed, r, 1])
    return disk_collision(n, gals, seeds, device, precision=precision)


def ensemble_sizes(nruns=48, base_seed=1311):
    """Grid size of each ensemble member without building its fields."""
    out = []
    for r in range(nruns):
        rng = np.random.Generator(np.random.PCG64([base_seed, r]))
        out.append(int(rng.choice([64, 96, 128])))
    return out


# --------------------------------------------------------------------------
# Verification problems of Sec. 4 of the paper

SHOCK_TUBES = {
    # (rho_L, v_L, p_L, rho_R, v_R, p_R, t_end): Table "ShockTube"
    1: (2.0, 0.0, 2.0, 1.0, 0.0, 1.0, 0.2),
    2: (1.0, -2.0, 0.4, 1.0, 2.0, 0.4, 0.15),
    3: (1.0, 0.0, 1000.0, 1.0, 0.0, 0.01, 0.012),
}


def _tube_config(n, axis, transverse=4, gamma=1.4, t_end=0.0, cfl=0.2, eta=1e-3):
    nn = [transverse] * 3
    nn[axis] = n
    h = 1.0 / n
    lo = [0.0] * 3
    hi = [transverse * h] * 3
    hi[axis] = 1.0
    bc = [1, 1, 1]
    bc[axis] = 0
    return base_config(tuple(nn), lo=tuple(lo), hi=tuple(hi), gamma=gamma, G=0.0,
                       cfl=cfl, eta=eta, bc=tuple(bc), t_end=t_end)


def gas_shock_tube(test, n=256, axis=0, transverse=4, gamma=1.4, device="cpu", eta=1e-3):
    """Gas tube of Table "ShockTube" along `axis`, x0 = 0.5, gamma = 1.4.  The
    BME component is a passive, uniform, static background."""
    rl, vl, pl, rr, vr, pr, t_end = SHOCK_TUBES[test]
    cfg = _tube_config(n, axis, transverse, gamma, t_end, eta=eta)
    X = cell_centres(cfg, device)[axis]
    left = X <= 0.5
    one = torch.ones_like(X)
    zero = torch.zeros_like(X)
    rho = torch.where(left, rl * one, rr * one)
    p = torch.where(left, pl * one, pr * one)
    vn = torch.where(left, vl * one, vr * one)
    v = [zero, zero, zero]
    v[axis] = vn
    Pi = [one, zero, zero, one.clone(), zero, one.clone()]
    return cfg, assemble(rho, v, p, one.clone(), [zero] * 3, Pi, gamma)


def bme_shock_tube(n=256, axis=0, transverse=4, t_end=0.2, device="cpu", eta=1e-3,
                   left_state=(2.0, 2.0), right_state=(1.0, 1.0)):
    """Shock tube of Sec. 4.2 for the moment equations: left state n = 2,
    Pi = diag-like [2,1,1;1,1,1] (Pi_dd = 2, all other components 1), right
    state n = 1, all Pi components 1, u = 0.  The normal axis plays x.
    left_state / right_state = (n, Pi_dd) on each side; every other stress
    component is 1."""
    cfg = _tube_config(n, axis, transverse, 1.4, t_end, eta=eta)
    X = cell_centres(cfg, device)[axis]
    left = X <= 0.5
    one = torch.ones_like(X)
    zero = torch.zeros_like(X)
    nb = torch.where(left, left_state[0] * one, right_state[0] * one)
    pdd = torch.where(left, left_state[1] * one, right_state[1] * one)
    Pi = [one.clone() for _ in range(6)]
    Pi[[0, 3, 5][axis]] = pdd
    # passive uniform gas
    gas_p = one.clone()
    return cfg, assemble(one.clone(), [zero] * 3, gas_p, nb, [zero] * 3, Pi, 1.4)


def aksenov(n=128, transverse=4, device="cpu", eta=1e-3):
    """Aksenov test (Sec. 4.3): gamma = 3, p = rho^3 (p0 = rho0 = 1), periodic on
    [0, 2 pi], rho = 1 + 0.5 cos x, u = 0.  Dimensionless time t' = pi/2 is the
    physical time pi / (2 sqrt 3)."""
    L = 2.0 * math.pi
    h = L / n
    cfg = base_config((n, transverse, transverse), lo=(0.0, 0.0, 0.0),
                      hi=(L, transverse * h, transverse * h), gamma=3.0, G=0.0,
                      bc=(1, 1, 1), t_end=math.pi / (2.0 * math.sqrt(3.0)), eta=eta)
    X = cell_centres(cfg, device)[0]
    rho = 1.0 + 0.5 * torch.cos(X)
    zero = torch.zeros_like(X)
    one = torch.ones_like(X)
    p = rho ** 3
    Pi = [one, zero, zero, one.clone(), zero, one.clone()]
    return cfg, assemble(rho, [zero] * 3, p, one.clone(), [zero] * 3, Pi, 3.0)


def random_periodic(n=(16, 12, 8), seed=0, device="cpu", amp=0.3, G=1.0, lo=-1.0, noise=0.01):
    """Smooth random periodic state with both components moving, for
    conservation and parity checks on non-cubic, non-power-of-two grids."""
    if isinstance(n, int):
        n = (n, n, n)
    h = 2.0 / n[0]
    cfg = base_config(n, lo=(lo,) * 3, hi=tuple(lo + h * v for v in n), G=G, bc=(1, 1, 1))
    shape = (n[2], n[1], n[0])
    X, Y, Z = cell_centres(cfg, device)
    k = [2.0 * math.pi / (h * v) for v in n]
    rng = np.random.Generator(np.random.PCG64(seed))
    ph = rng.uniform(0, 2 * math.pi, 20)

    def mode(i, a):
        return a * torch.sin(k[0] * X + ph[i]) * torch.cos(k[1] * Y + ph[i + 1]) * torch.sin(k[2] * Z + ph[i + 2] + 0.3)

    rho = 1.0 + mode(0, amp) + noise * normal_noise(seed + 1000, shape, device)
    nb = 1.0 + mode(1, amp) + noise * normal_noise(seed + 2000, shape, device)
    v = [mode(2 + i, 0.4) for i in range(3)]
    u = [mode(5 + i, 0.4) for i in range(3)]
    p = 0.5 + mode(8, 0.2)
    diag = [0.4 + mode(9 + i, 0.1) for i in range(3)]
    off = [mode(12 + i, 0.05) for i in range(3)]
    Pi = [diag[0], off[0], off[1], diag[1], off[2], diag[2]]
    return cfg, assemble(rho, v, p, nb, u, Pi, cfg["gamma"])


def hydrostatic_sphere(n=32, L=2.0, device="cpu", floor=1e-3):
    """Gas sphere rho0 = 1 - r in hydrostatic equilibrium with the closed-form
    pressure p0(r) of Sec. 4.5 (G = 1), on [-L, L]^3; the stars/dark-matter
    component is a cold, static trace.  Density and pressure are floored
    outside r = 1."""
    cfg = base_config(n, lo=-L, hi=L, G=1.0)
    X, Y, Z = cell_centres(cfg, device)
    r = torch.sqrt(X * X + Y * Y + Z * Z)
    inside = r <= 1.0
    rho = torch.where(inside, 1.0 - r, torch.zeros_like(r)).clamp(min=floor)
    p0 = -(math.pi * r * r / 36.0) * (9 * r * r - 28 * r + 24) + 5 * math.pi / 36.0
    p = torch.where(inside, p0, torch.zeros_like(r)).clamp(min=floor * 0.1)
    zero = torch.zeros_like(r)
    tiny = torch.full_like(r, 1e-6)
    Pi = [tiny * 1e-3, zero, zero, tiny * 1e-3, zero, tiny * 1e-3]
    return cfg, assemble(rho, [zero] * 3, p, tiny, [zero] * 3, Pi, cfg["gamma"])


# --------------------------------------------------------------------------
# Instability tests (Sec. 4.4) and the author's cloud collision (Sec. 4.5)

def _plane_config(n, nz, gamma, bc, G=0.0):
    """[-0.5, 0.5]^2 in x, y on n x n cells; nz cells of the same size along a
    periodic z (the two-dimensional tests run on a thin slab)."""
    h = 1.0 / n
    return base_config((n, n, nz), lo=(-0.5, -0.5, -0.5 * nz * h), hi=(0.5, 0.5, 0.5 * nz * h),
                       gamma=gamma, G=G, bc=bc)


def _cold_trace(like):
    """Stars / dark matter as a cold, static trace (these tests are gas only)."""
    zero = torch.zeros_like(like)
    tiny = torch.full_like(like, 1e-6)
    return tiny, [zero] * 3, [tiny * 1e-3, zero, zero, tiny * 1e-3, zero, tiny * 1e-3]


def kelvin_helmholtz(n=128, nz=4, device="cpu", gamma=1.4):
    """Kelvin-Helmholtz instability of Sec. 4.4 on [-0.5, 0.5]^2, periodic on
    every axis, gamma = 1.4, p = 2.5, no gravity.  v_x = 0.5 in the band
    |y| <= 0.25 and -0.5 outside; v_y = A(y) (1 + cos 8 pi x)(1 + cos 8 pi y)
    with A = 0.01 where ||y| - 0.25| <= 0.01, else 0.  The printed density
    repeats the Rayleigh-Taylor one with a garbled argument; the reading is
    density 2 in the band and 1 outside."""
    cfg = _plane_config(n, nz, gamma, (1, 1, 1))
    X, Y, _ = cell_centres(cfg, device)
    band = Y.abs() <= 0.25
    one = torch.ones_like(X)
    rho = torch.where(band, 2.0 * one, one)
    vx = torch.where(band, 0.5 * one, -0.5 * one)
    A = torch.where(((Y.abs() - 0.25).abs() <= 0.01), 0.01 * one, 0.0 * one)
    vy = A * (1.0 + torch.cos(8.0 * math.pi * X)) * (1.0 + torch.cos(8.0 * math.pi * Y))
    nb, u, Pi = _cold_trace(X)
    return cfg, assemble(rho, [vx, vy, torch.zeros_like(X)], 2.5 * one, nb, u, Pi, gamma)


def rayleigh_taylor(n=128, nz=4, device="cpu", gamma=1.4, g=0.1):
    """Rayleigh-Taylor instability of Sec. 4.4 on [-0.5, 0.5]^2, gamma = 1.4:
    density 1 for y <= 0 and 2 above, the hydrostatic pressure
    p = 2.5 - rho g y under a uniform downward gravity g (not printed; the
    reading is 0.1), v_y = A(y) (1 + cos 2 pi x)(1 + cos 2 pi y) with A = 0.01
    where |y| <= 0.01, else 0.  Periodic in x and z, outflow in y, no
    self-gravity; the field enters as the external acceleration (0, -g, 0)."""
    cfg = _plane_config(n, nz, gamma, (1, 0, 1))
    cfg["gext"] = (0.0, -g, 0.0)
    X, Y, _ = cell_centres(cfg, device)
    one = torch.ones_like(X)
    rho = torch.where(Y <= 0.0, one, 2.0 * one)
    p = 2.5 - rho * g * Y
    A = torch.where(Y.abs() <= 0.01, 0.01 * one, 0.0 * one)
    vy = A * (1.0 + torch.cos(2.0 * math.pi * X)) * (1.0 + torch.cos(2.0 * math.pi * Y))
    zero = torch.zeros_like(X)
    nb, u, Pi = _cold_trace(X)
    return cfg, assemble(rho, [zero, vy, zero], p, nb, u, Pi, gamma)


def sphere_profile(r):
    """The hydrostatic gas sphere of Sec. 4.5 (G = 1): density 1 - r,
    pressure p0(r) and potential Phi0(r) inside r <= 1; 0, 0 and -pi / (3 r)
    outside."""
    inside = r <= 1.0
    zero = torch.zeros_like(r)
    rho = torch.where(inside, 1.0 - r, zero)
    p = torch.where(inside, -(math.pi * r * r / 36.0) * (9 * r * r - 28 * r + 24) + 5 * math.pi / 36.0, zero)
    phi = torch.where(inside, -(math.pi / 3.0) * (r ** 3 - 2 * r * r) - 2 * math.pi / 3.0,
                      -math.pi / (3.0 * r.clamp(min=1e-12)))
    return rho, p, phi


def cloud_collision(n=(96, 64, 64), device="cpu", L0=2.4, v_collide=1.0, floor=1e-3, poisson="isolated",
                    precision="fp64"):
    """The author's cloud collision of Sec. 4.5: two hydrostatic spheres
    (density 1 - r, pressure p0(r); G = 1) whose centres start L0 = 2.4 apart
    on the x axis and close at v_collide = 1 (each moving at 1/2).  Reading:
    domain [-2.4, 2.4] x [-1.6, 1.6]^2 (cubic cells for the default n),
    gamma = 5/3, density and pressure floored outside the spheres (1e-3 and
    1e-4), isolated potential; the stars / dark matter are a cold static
    trace.  The setup is mirror-symmetric in x."""
    h = 4.8 / n[0]
    cfg = base_config(n, lo=(-2.4, -0.5 * n[1] * h, -0.5 * n[2] * h), hi=(2.4, 0.5 * n[1] * h, 0.5 * n[2] * h),
                      G=1.0, poisson=poisson, precision=precision)
    X, Y, Z = cell_centres(cfg, device)
    rho = torch.zeros_like(X)
    p = torch.zeros_like(X)
    mom = torch.zeros_like(X)
    for cx, vx in ((-0.5 * L0, 0.5 * v_collide), (0.5 * L0, -0.5 * v_collide)):
        r = torch.sqrt((X - cx) ** 2 + Y * Y + Z * Z)
        rs, ps, _ = sphere_profile(r)
        rho = rho + rs
        p = p + ps
        mom = mom + rs * vx
    rho = rho.clamp(min=floor)
    vx = mom / rho
    p = p.clamp(min=floor * 0.1)
    zero = torch.zeros_like(X)
    nb, u, Pi = _cold_trace(X)
    return cfg, assemble(rho, [vx, zero, zero], p, nb, u, Pi, cfg["gamma"])


def to_numpy(state):
    return {k: v.detach().cpu().numpy() for k, v in state.items()}
