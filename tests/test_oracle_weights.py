"""Pins of the oracle's time-stepping weights against exact mathematics.

Sec. 3.2.2.1 (Eq. 23-30), Sec. 3.2.2.2 (Eq. 31-41), Sec. 3.2.2.3 (Eq. 42-46),
Sec. 3.2.2.4 (Eq. 47) of arXiv 1909.04153.  Every expected value here comes
from exact rational arithmetic (fractions) on the defining polynomials, not
from the printed formulas.
"""
import math
import random
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import oracle as O


def _poly_mul(a, b):
    out = [Fr(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _lagrange_basis(nodes, j):
    """coefficients (ascending powers of t) of the Lagrange basis polynomial j"""
    p = [Fr(1)]
    for k, tk in enumerate(nodes):
        if k != j:
            p = _poly_mul(p, [-tk / (nodes[j] - tk), Fr(1) / (nodes[j] - tk)])
    return p


def _integrate(p, a, b):
    return sum(c * (b ** (k + 1) - a ** (k + 1)) / (k + 1) for k, c in enumerate(p))


def _evaluate(p, t):
    return sum(c * t ** k for k, c in enumerate(p))


def _derivative(p):
    return [c * k for k, c in enumerate(p)][1:]


def _nodes(h1, h2):
    # t_n = 0, t_{n-1} = -h1, t_{n-2} = -(h1 + h2)
    return [Fr(0), -h1, -(h1 + h2)]


def _rand_steps(rng):
    return [Fr(rng.randint(1, 97), rng.randint(1, 97)) for _ in range(3)]


def test_ab3_constant_step_collapse():
    # Sec. 3.2.2.1: equal steps give 23/12, -16/12, 5/12
    for h in (1.0, 0.37, 2.5e-3):
        a = O.ab3_alpha(h, h, h)
        np.testing.assert_allclose(a * 12.0 / h, [23.0, -16.0, 5.0], rtol=0, atol=1e-13)


def test_ab3_equals_integral_of_lagrange_interpolant():
    rng = random.Random(1)
    for _ in range(50):
        h0, h1, h2 = _rand_steps(rng)
        nodes = _nodes(h1, h2)
        exact = [_integrate(_lagrange_basis(nodes, j), Fr(0), h0) for j in range(3)]
        got = O.ab3_alpha(float(h0), float(h1), float(h2))
        np.testing.assert_allclose(got, [float(e) for e in exact], rtol=1e-13, atol=1e-15)


def test_ab3_exact_on_quadratics_and_sums_to_step():
    rng = random.Random(2)
    for _ in range(20):
        h0, h1, h2 = (float(v) for v in _rand_steps(rng))
        a = O.ab3_alpha(h0, h1, h2)
        t = np.array([0.0, -h1, -(h1 + h2)])
        for p, integral in ((0, h0), (1, h0 ** 2 / 2), (2, h0 ** 3 / 3)):
            assert abs(np.dot(a, t ** p) - integral) <= 1e-12 * max(1.0, abs(integral))


def test_ab3_third_order_on_ode_with_variable_steps():
    """X' = cos(t) integrated with exact history and a variable step pattern;
    the global error shrinks like h^3."""
    def run(h):
        ratios = [1.0, 1.3, 0.8, 1.1, 0.9]
        ts = [0.0, h, 2.2 * h]
        X = [math.sin(t) for t in ts]
        k = 0
        while ts[-1] < 2.0:
            h0 = ratios[k % 5] * h
            h1, h2 = ts[-1] - ts[-2], ts[-2] - ts[-3]
            a = O.ab3_alpha(h0, h1, h2)
            f = [math.cos(ts[-1]), math.cos(ts[-2]), math.cos(ts[-3])]
            X.append(X[-1] + a[0] * f[0] + a[1] * f[1] + a[2] * f[2])
            ts.append(ts[-1] + h0)
            k += 1
        return abs(X[-1] - math.sin(ts[-1])) / ts[-1]
    e = [run(0.02 / 2 ** k) for k in range(4)]
    orders = [math.log2(e[k] / e[k + 1]) for k in range(3)]
    assert all(2.8 < o < 3.2 for o in orders), orders


def test_fd_weights_special_cases():
    # Sec. 3.2.2.2: BDF2 at t_i, central at t_{i-1}, forward at t_{i-2}
    h = 0.25
    D = O.fd_weights(h, h) * h
    np.testing.assert_allclose(D[0], [1.5, -2.0, 0.5], atol=1e-14)
    np.testing.assert_allclose(D[1], [0.5, 0.0, -0.5], atol=1e-14)
    np.testing.assert_allclose(D[2], [-0.5, 2.0, -1.5], atol=1e-14)


def test_fd_weights_exact_on_quadratics():
    rng = random.Random(3)
    for _ in range(50):
        _, h1, h2 = _rand_steps(rng)
        nodes = _nodes(h1, h2)
        D = O.fd_weights(float(h1), float(h2))
        for p in range(3):
            Y = [float(t ** p) for t in nodes]
            for k in range(3):
                exact = float(p * nodes[k] ** (p - 1)) if p > 0 else 0.0
                assert abs(np.dot(D[k], Y) - exact) <= 1e-11 * max(1.0, abs(exact))


def test_fstar_weights_are_quadratic_extrapolation():
    """Eq. 43 with Eq. 44-46 composes to the increment of the quadratic
    interpolant of F* through the last three levels, evaluated at t_{n+1}."""
    rng = random.Random(4)
    for _ in range(50):
        h0, h1, h2 = _rand_steps(rng)
        nodes = _nodes(h1, h2)
        exact = [_evaluate(_lagrange_basis(nodes, j), h0) - (1 if j == 0 else 0) for j in range(3)]
        a, D = O.step_weights(5, float(h0), float(h1), float(h2))
        beta = a @ D
        np.testing.assert_allclose(beta, [float(e) for e in exact], rtol=1e-12, atol=1e-13)
    a, D = O.step_weights(5, 0.1, 0.1, 0.1)
    np.testing.assert_allclose(a @ D, [2.0, -3.0, 1.0], atol=1e-13)  # Eq. 17


def test_bootstrap_and_linear_reading_weights():
    a, D = O.step_weights(0, 0.3, 0.0, 0.0)
    np.testing.assert_array_equal(a, [0.3, 0.0, 0.0])
    assert not np.any(a @ D)
    a, D = O.step_weights(1, 0.3, 0.2, 0.0)
    np.testing.assert_allclose(a, [0.3, 0.0, 0.0])
    np.testing.assert_allclose(a @ D, [1.5, -1.5, 0.0], atol=1e-15)
    # linear reading: increment of the line through the last two levels
    rng = random.Random(5)
    for _ in range(20):
        h0, h1, h2 = (float(v) for v in _rand_steps(rng))
        a, D = O.step_weights(7, h0, h1, h2, fstar_order=1)
        np.testing.assert_allclose(a @ D, [h0 / h1, -h0 / h1, 0.0], rtol=1e-13, atol=1e-15)


def test_lazy_ema_sequences():
    a = 0.1
    # drops are taken at once
    assert O.lazy_ema(0.5, 1.0, a) == 0.5
    assert O.lazy_ema(1.0, 1.0, a) == 1.0
    # rises close the gap geometrically
    prev, cand = 1.0, 2.0
    seq = []
    for _ in range(30):
        prev = O.lazy_ema(cand, prev, a)
        seq.append(prev)
    gaps = [cand - s for s in seq]
    np.testing.assert_allclose(gaps, [0.9 ** (k + 1) for k in range(30)], rtol=1e-12)
    assert all(s < cand for s in seq)
