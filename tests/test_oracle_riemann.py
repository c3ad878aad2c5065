"""Pins of the oracle's interface (Riemann) states, Sec. 2.1 and 2.2.

The closed forms printed in the paper are the exact solutions of linear
hyperbolic systems with frozen coefficients.  Here the exact linear Riemann
solution is built independently with the matrix sign function of the printed
system matrix, q* = (qL + qR)/2 - sign(M) (qR - qL)/2, and compared with the
oracle's closed form."""
import numpy as np
import pytest


def msign(M):
    w, V = np.linalg.eig(M)
    return np.real(V @ np.diag(np.sign(np.real(w))) @ np.linalg.inv(V))


def linear_riemann(M, qL, qR):
    return 0.5 * (qL + qR) - 0.5 * msign(M) @ (qR - qL)


def test_gas_face_is_exact_linear_solution(orc):
    rng = np.random.default_rng(11)
    for _ in range(50):
        rl, rr = rng.uniform(0.1, 3.0, 2)
        pl, pr = rng.uniform(0.05, 5.0, 2)
        vl, vr = rng.normal(size=2)
        g = rng.uniform(1.1, 3.0)
        # (v, p) system of Sec. 2.1 with the density row removed; the closed
        # form corresponds to the mean pressure and the harmonic-mean density
        rt = 2.0 * rl * rr / (rl + rr)
        pt = 0.5 * (pl + pr)
        M = np.array([[0.0, 1.0 / rt], [g * pt, 0.0]])
        ref = linear_riemann(M, np.array([vl, pl]), np.array([vr, pr]))
        V, P = orc.riemann_gas(rl, vl, pl, rr, vr, pr, g)
        np.testing.assert_allclose([V, P], ref, rtol=1e-12, atol=1e-13)


def test_gas_face_special_cases(orc):
    # equal states: no wave, the state itself
    V, P = orc.riemann_gas(1.3, 0.7, 2.1, 1.3, 0.7, 2.1, 1.4)
    assert V == pytest.approx(0.7, abs=1e-15) and P == pytest.approx(2.1, rel=1e-15)
    # mirror: swap sides and flip the normal velocity
    a = orc.riemann_gas(1.0, 0.3, 1.0, 0.5, -0.2, 0.4, 1.4)
    b = orc.riemann_gas(0.5, 0.2, 0.4, 1.0, -0.3, 1.0, 1.4)
    assert a[0] == pytest.approx(-b[0], abs=1e-15) and a[1] == pytest.approx(b[1], rel=1e-15)
    # pure pressure jump at rest: acoustic impedance Z = sqrt(gamma p rho)
    V, P = orc.riemann_gas(1.0, 0.0, 1.0 + 1e-6, 1.0, 0.0, 1.0 - 1e-6, 1.4)
    assert V == pytest.approx(1e-6 / np.sqrt(1.4), rel=1e-6)


def bme_matrix(n, A, B, C):
    """6x6 Eulerian-stage BME matrix of Sec. 2.2 for q = (u_d, u_a, u_b,
    Pi_dd, Pi_da, Pi_db)."""
    M = np.zeros((6, 6))
    M[0, 3] = M[1, 4] = M[2, 5] = 1.0 / n
    M[3, 0] = 3.0 * A
    M[4, 0] = 2.0 * B
    M[4, 1] = A
    M[5, 0] = 2.0 * C
    M[5, 2] = A
    return M


SYM = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}


def sym(i, j):
    return SYM[(min(i, j), max(i, j))]


@pytest.mark.parametrize("d", [0, 1, 2])
def test_bme_face_is_exact_linear_solution(orc, d):
    rng = np.random.default_rng(100 + d)
    a, b = (d + 1) % 3, (d + 2) % 3
    for _ in range(40):
        nl, nr = rng.uniform(0.2, 3.0, 2)
        ul, ur = rng.normal(size=3), rng.normal(size=3)
        pil = rng.uniform(-0.3, 0.3, 6)
        pir = rng.uniform(-0.3, 0.3, 6)
        for i in range(3):
            pil[sym(i, i)] = rng.uniform(0.5, 3.0)
            pir[sym(i, i)] = rng.uniform(0.5, 3.0)
        us, ps = orc.riemann_bme(nl, ul, pil, nr, ur, pir, d)
        nbar = 0.5 * (nl + nr)
        A = 0.5 * (pil[sym(d, d)] + pir[sym(d, d)])
        B = 0.5 * (pil[sym(d, a)] + pir[sym(d, a)])
        C = 0.5 * (pil[sym(d, b)] + pir[sym(d, b)])
        M = bme_matrix(nbar, A, B, C)
        qL = np.array([ul[d], ul[a], ul[b], pil[sym(d, d)], pil[sym(d, a)], pil[sym(d, b)]])
        qR = np.array([ur[d], ur[a], ur[b], pir[sym(d, d)], pir[sym(d, a)], pir[sym(d, b)]])
        ref = linear_riemann(M, qL, qR)
        got = np.array([us[d], us[a], us[b], ps[d], ps[a], ps[b]])
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12)


def test_bme_face_equal_states(orc):
    u = np.array([0.1, -0.2, 0.3])
    pi = np.array([1.5, 0.2, -0.1, 0.9, 0.05, 1.2])
    for d in range(3):
        us, ps = orc.riemann_bme(1.7, u, pi, 1.7, u, pi, d)
        np.testing.assert_allclose(us, u, rtol=0, atol=1e-15)
        np.testing.assert_allclose(ps, [pi[sym(d, 0)], pi[sym(d, 1)], pi[sym(d, 2)]], rtol=1e-15)


def test_bme_eigenvalues_match_paper(orc):
    """The printed eigenvalues +-sqrt(3 Pi_xx / rho), +-sqrt(Pi_xx / rho) (twice)."""
    M = bme_matrix(1.3, 0.7, 0.2, -0.1)
    w = np.sort(np.real(np.linalg.eigvals(M)))
    c1, c2 = np.sqrt(3 * 0.7 / 1.3), np.sqrt(0.7 / 1.3)
    np.testing.assert_allclose(w, [-c1, -c2, -c2, c2, c2, c1], rtol=1e-6)
