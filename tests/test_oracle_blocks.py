"""Pins of the oracle's building blocks: the tridiagonal solve of Eq. 19-21,
the generalised minmod, the KP07 central-upwind face flux (reading of Sec.
3.1) and the Madsen-Sorensen wave number used by the wavemaker."""
import math

import numpy as np
import pytest

from oracle import oracle as O

G = 9.81


def test_thomas_matches_dense_solve():
    rng = np.random.default_rng(0)
    for n in (3, 7, 32, 64):
        k = rng.uniform(0.0, 200.0, n)
        s = rng.uniform(-1.0, 1.0, n) * 0.3 * k
        a, c = s - k, -s - k          # Eq. 21 shape: A = s - k, C = -s - k
        b = 1.0 + 2.0 * k
        r = rng.normal(size=n)
        M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        x_ref = np.linalg.solve(M, r)
        x = O.thomas(a, b, c, r)
        assert np.max(np.abs(M @ x - r)) <= 1e-12 * np.max(np.abs(r)) * np.max(b)
        np.testing.assert_allclose(x, x_ref, rtol=1e-12, atol=1e-14)


def _thomas_extended(a, b, c, r):
    # the same elimination in numpy's extended precision (80-bit on x86-64)
    a, b, c, r = (np.asarray(v, dtype=np.longdouble) for v in (a, b, c, r))
    n = len(r)
    cp = np.zeros(n, dtype=np.longdouble)
    rp = np.zeros(n, dtype=np.longdouble)
    cp[0], rp[0] = c[0] / b[0], r[0] / b[0]
    for i in range(1, n):
        m = b[i] - a[i] * cp[i - 1]
        cp[i], rp[i] = c[i] / m, (r[i] - a[i] * rp[i - 1]) / m
    x = np.zeros(n, dtype=np.longdouble)
    x[-1] = rp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = rp[i] - cp[i] * x[i + 1]
    return x


def test_line_solve_reaches_the_exact_solution_on_long_lines():
    # Eq. 19-21 on a 2100-cell line at d/dx = 20 ((B + 1/3) d^2/dx^2 = 160,
    # condition number ~641), wall folds at both ends, a smooth wave plus
    # noise on the right-hand side: the plain FP64 sweep is ~1e-14 off the
    # extended-precision solution; the step's refined solve must be at
    # FP64 rounding of it
    if np.finfo(np.longdouble).eps > 1e-18:
        pytest.skip("no extended precision long double on this host")
    n, k = 2100, (1.0 / 15.0 + 1.0 / 3.0) * 400.0
    a = np.full(n, -k)
    c = np.full(n, -k)
    b = np.full(n, 1.0 + 2.0 * k)
    b[0] -= a[0]
    b[-1] -= c[-1]
    a[0] = c[-1] = 0.0
    rng = np.random.default_rng(1)
    x0 = np.arange(n) * 0.05
    r = 0.1 * np.exp(-((x0 - 50.0) / 1.0) ** 2) + 1e-3 * rng.normal(size=n)
    xe = _thomas_extended(a, b, c, r)
    rel = lambda x: float(np.linalg.norm((x - xe).astype(np.float64)) / np.linalg.norm(xe.astype(np.float64)))
    assert rel(O.solve_line(a, b, c, r)) <= 2e-16
    assert rel(O.thomas(a, b, c, r)) >= 1e-15   # the refinement is what closes the gap


def test_minmod():
    assert O.minmod(1.0, 2.0, 3.0) == 1.0
    assert O.minmod(-1.0, -2.0, -0.5) == -0.5
    assert O.minmod(1.0, -2.0, 3.0) == 0.0
    assert O.minmod(0.0, 2.0, 3.0) == 0.0


def test_face_flux_uniform_state_is_physical_flux():
    h, P, Q = 0.8, 0.3, -0.2
    H = O.face_flux_const(h, P, Q, h, P, Q, bf=0.0, eps=1e-12)
    np.testing.assert_allclose(H, [P, P * P / h + 0.5 * G * h * h, P * Q / h], rtol=1e-13)


def test_face_flux_lake_at_rest_is_hydrostatic():
    for bf in (-1.0, -0.3, 0.2):
        w = 0.5
        H = O.face_flux_const(w, 0.0, 0.0, w, 0.0, 0.0, bf=bf, eps=1e-12)
        h = w - bf
        np.testing.assert_allclose(H, [0.0, 0.5 * G * h * h, 0.0], rtol=1e-14, atol=1e-15)


def test_face_flux_dry_and_mirror():
    np.testing.assert_array_equal(O.face_flux_const(0.0, 0.0, 0.0, 0.0, 0.0, 0.0, bf=0.0), [0.0, 0.0, 0.0])
    # a wall is a mirror: (w, P, Q) | (w, -P, Q) carries no mass
    H = O.face_flux_const(0.7, 0.25, 0.1, 0.7, -0.25, 0.1, bf=-0.3, eps=1e-12)
    assert H[0] == 0.0
    # left-right reflection flips the mass flux sign, keeps the momentum flux
    H1 = O.face_flux_const(0.9, 0.4, 0.05, 0.6, 0.1, -0.02, bf=-0.2, eps=1e-12)
    H2 = O.face_flux_const(0.6, -0.1, -0.02, 0.9, -0.4, 0.05, bf=-0.2, eps=1e-12)
    np.testing.assert_allclose([H1[0], H1[1]], [-H2[0], H2[1]], rtol=1e-13)


def test_ms_wavenumber_solves_linear_dispersion():
    B = 1.0 / 15.0
    for d in (0.5, 1.0, 8.0):
        for T in (1.0, 2.0, 8.0, 20.0):
            om = 2.0 * math.pi / T
            k = O.ms_wavenumber(om, d, G, B)
            kd = k * d
            w2 = G * d * k * k * (1 + B * kd * kd) / (1 + (B + 1.0 / 3.0) * kd * kd)
            assert abs(w2 - om * om) <= 1e-12 * om * om
    # shallow-water limit
    k = O.ms_wavenumber(2 * math.pi / 1000.0, 1.0, G, B)
    assert abs(k - 2 * math.pi / 1000.0 / math.sqrt(G)) < 1e-6 * k
