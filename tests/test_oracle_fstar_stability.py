"""Linear stability of the constant-step scheme in 2D: amplification matrix
from the Fourier symbols of the discrete operators, checked against the
oracle's own growth of single modes.

Linearised about a lake at rest on a flat bed of depth d (central slopes,
theta = 0, so the reconstruction is linear; c = sqrt(g d)):
  * KP07 central-upwind fluxes (Sec. 3.1, Eq. 11-13) reduce to the average
    of the two face states' physical fluxes minus (c/2) times their jump;
  * the dispersive terms of Eq. 12-13 and F*, G* of Eq. 14-15 are the
    oracle's central stencils;
  * U* = T_x P, V* = T_y Q with the Eq. 21 coefficients;
  * constant-step AB3 (Eq. 16) for E, F, G, and the F*, G* increment by
    quadratic extrapolation (2, -3, 1; Eq. 17) or, in the linear reading,
    by the last difference (1, -1, 0).
The state (eta, P, Q) and its two previous levels form a 9-vector per
Fourier mode; the step is a 9 x 9 matrix whose spectral radius is the
mode's growth per step.

Findings, each pinned below:
  * quadratic extrapolation grows at every CFL number once d / dx >= 2
    (about 1.26 per step at d / dx = 2, 1.84 at 5, 2.10 at 10): the cross
    terms (B + 1/3) d^2 P_xy, Q_xy couple P and Q through an explicit
    second-order extrapolation whose ratio to the implicit operator exceeds
    1/3 for modes with k d above about 1;
  * the linear reading is stable up to CFL 6/11/4 = 0.136 (the AB3 stability
    interval on the negative real axis against the 2D checkerboard mode's
    damping -4 CFL), the limit seen on 2D runs;
  * the oracle grows single wall-compatible modes at exactly these rates.
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleDomain
from paper_1909_04153_amd import scenarios as S

G, B = 9.81, 1.0 / 15.0


def step_matrix(tx, ty, d, dx, dy, dt, order):
    c = math.sqrt(G * d)
    cb = (B + 1.0 / 3.0) * d * d
    ex, ey = np.exp(1j * tx), np.exp(1j * ty)
    sx, sy = math.sin(tx), math.sin(ty)
    # face states at i+1/2 of a mode e^{i theta i}: left = cell i + slope / 2,
    # right = cell i+1 - slope / 2, central slope (q_{i+1} - q_{i-1}) / 2
    lx, rx = 1.0 + 0.5j * sx, ex * (1.0 - 0.5j * sx)
    ly, ry = 1.0 + 0.5j * sy, ey * (1.0 - 0.5j * sy)
    avx, jx, avy, jy = 0.5 * (lx + rx), rx - lx, 0.5 * (ly + ry), ry - ly
    dfx, dfy = (1.0 - 1.0 / ex) / dx, (1.0 - 1.0 / ey) / dy     # face difference over a cell
    L = np.zeros((3, 3), complex)                               # (E, F, G) <- (eta, P, Q)
    # x-faces: mass flux P, normal momentum g d eta, tangential 0; jumps of eta, P, Q
    L[0, 0] -= -0.5 * c * jx * dfx
    L[0, 1] -= avx * dfx
    L[1, 0] -= G * d * avx * dfx
    L[1, 1] -= -0.5 * c * jx * dfx
    L[2, 2] -= -0.5 * c * jx * dfx
    # y-faces
    L[0, 0] -= -0.5 * c * jy * dfy
    L[0, 2] -= avy * dfy
    L[1, 1] -= -0.5 * c * jy * dfy
    L[2, 0] -= G * d * avy * dfy
    L[2, 2] -= -0.5 * c * jy * dfy
    # dispersive terms of Eq. 12-13 on a flat bed
    d2x, d2y = ex - 2.0 + 1.0 / ex, ey - 2.0 + 1.0 / ey
    exxx = (ex ** 2 - 2.0 * ex + 2.0 / ex - ex ** -2) / (2.0 * dx ** 3)
    eyyy = (ey ** 2 - 2.0 * ey + 2.0 / ey - ey ** -2) / (2.0 * dy ** 3)
    exyy = (ex - 1.0 / ex) * d2y / (2.0 * dx * dy * dy)
    exxy = (ey - 1.0 / ey) * d2x / (2.0 * dx * dx * dy)
    L[1, 0] += B * G * d ** 3 * (exxx + exyy)
    L[2, 0] += B * G * d ** 3 * (eyyy + exxy)
    # F* = (B + 1/3) d^2 Q_xy, G* = (B + 1/3) d^2 P_xy (Eq. 14-15, flat bed)
    sxy = cb * (ex - 1.0 / ex) * (ey - 1.0 / ey) / (4.0 * dx * dy)
    Fs = np.zeros((3, 3), complex)
    Fs[1, 2] = Fs[2, 1] = sxy
    Tinv = np.diag([1.0, 1.0 / (1.0 - cb * d2x / dx ** 2), 1.0 / (1.0 - cb * d2y / dy ** 2)])
    alpha = dt * np.array([23.0, -16.0, 5.0]) / 12.0
    beta = np.array([2.0, -3.0, 1.0]) if order == 2 else np.array([1.0, -1.0, 0.0])
    M = np.zeros((9, 9), complex)
    for k in range(3):
        M[0:3, 3 * k:3 * k + 3] = Tinv @ (alpha[k] * L + beta[k] * Fs)
    M[0:3, 0:3] += np.eye(3)
    M[3:6, 0:3] = np.eye(3)
    M[6:9, 3:6] = np.eye(3)
    return M


def rho(tx, ty, d_dx, cfl, order):
    dx = 1.0
    d = d_dx * dx
    return max(abs(np.linalg.eigvals(step_matrix(tx, ty, d, dx, dx, cfl * dx / math.sqrt(G * d), order))))


def worst(d_dx, cfl, order, n=24):
    th = np.linspace(math.pi / n, math.pi, n)
    return max(rho(a, b, d_dx, cfl, order) for a in th for b in th)


def test_symbol_matrix_reproduces_the_1d_scheme_limits():
    # a long 1D mode is neutral to rounding (AB3 on a nearly imaginary
    # eigenvalue); the 1D checkerboard is damped at CFL 0.2
    assert abs(rho(0.02, 1e-9, 5.0, 0.125, 2) - 1.0) < 1e-6
    assert rho(math.pi, 1e-9, 5.0, 0.2, 2) < 1.0


def test_quadratic_extrapolation_grows_in_2d_at_any_cfl():
    for d_dx, lo in ((2.0, 1.2), (5.0, 1.8), (10.0, 2.05)):
        for cfl in (0.02, 0.125):
            assert worst(d_dx, cfl, 2) > lo, (d_dx, cfl)
    # on grids coarse against the depth the same extrapolation is stable
    assert worst(1.0, 0.125, 2) <= 1.0 + 1e-9


def test_linear_reading_is_stable_up_to_the_ab3_limit():
    for d_dx in (0.5, 1.0, 2.0, 5.0, 10.0, 20.0):
        assert worst(d_dx, 0.125, 1) <= 1.0 + 1e-9, d_dx
        assert worst(d_dx, 0.13, 1) <= 1.0 + 1e-9, d_dx
        assert worst(d_dx, 0.14, 1) > 1.01, d_dx
    # the limit: AB3 is stable on [-6/11, 0] of the real axis, and the 2D
    # checkerboard mode is damped at -4 CFL per step
    lim = 6.0 / 11.0 / 4.0
    assert rho(math.pi, math.pi, 5.0, 0.999 * lim, 1) <= 1.0 + 1e-9
    assert rho(math.pi, math.pi, 5.0, 1.001 * lim, 1) > 1.0


@pytest.mark.parametrize("d_dx,cfl,order,m", [(5.0, 0.125, 2, 8), (10.0, 0.125, 2, 5), (2.0, 0.125, 2, 11),
                                              (1.0, 0.16, 1, 31)])
def test_oracle_grows_single_modes_at_the_predicted_rate(d_dx, cfl, order, m):
    """a wall-compatible mode eta = cos(th (i + 1/2)) cos(th (j + 1/2)),
    th = m pi / n, of amplitude 1e-10 d in a closed flat basin (fixed step,
    central slopes): its growth per step over steps 30..40 equals the
    spectral radius of the mode's step matrix"""
    n, dx = 32, 0.1
    d = d_dx * dx
    dt = cfl * dx / math.sqrt(G * d)
    p = S.base_params(n, n, dx, theta=0.0, fixed_dt=1, dt_init=dt, fstar_order=order)
    th = m * math.pi / n
    X, Y = S.cell_coords(n, n, dx, dx)
    eta = 1e-10 * d * np.cos(th * X / dx) * np.cos(th * Y / dx)
    o = OracleDomain(p, np.full((n + 1, n + 1), d))
    assert o.set_state(eta, 0.0 * eta, 0.0 * eta) == 0
    norms = []
    for k in range(40):
        assert o.step(1) == 0
        if k + 1 in (30, 40):
            norms.append(math.sqrt(sum(float(np.sum(o.read(f) ** 2)) for f in ("eta", "P", "Q"))))
    measured = (norms[1] / norms[0]) ** 0.1
    predicted = max(abs(np.linalg.eigvals(step_matrix(th, th, d, dx, dx, dt, order))))
    assert predicted > 1.1
    assert abs(measured - predicted) < 5e-3 * predicted, (measured, predicted)
