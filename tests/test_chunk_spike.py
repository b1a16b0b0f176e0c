"""The chunk solves of the stencil and finalize kernels split a chunk of a
line solve (Eq. 19-21) into P = 2 or 4 consecutive parts, one lane each:
every part is eliminated with zero coupling for the right-hand side and for
its two coupling columns, the parts' end values give a small system for the
unknowns at the part interfaces, and each part is corrected (the SPIKE
construction of the line coupling, applied inside the chunk).  This test
checks that construction, written out in numpy with the kernels' part sizes
(trailing parts empty when the chunk has fewer rows than lanes), against a
direct solve of the chunk's tridiagonal system, on matrices with the shape
of Eq. 21 (diagonal 1 + 2k, off-diagonals -k +/- s); and the finalize
kernel's two-vector form of the same construction for a right-hand side
with entries in the chunk's first and last rows only."""
import numpy as np
import pytest


def thomas_multi(a, b, c, R):
    """solve the tridiagonal system (a: sub, b: diag, c: super; a[0] and
    c[-1] unused) for the columns of R"""
    n = len(b)
    R = np.array(R, dtype=float)
    cp = np.zeros(n)
    u = b[0]
    R[0] /= u
    cp[0] = c[0] / u
    for k in range(1, n):
        u = b[k] - a[k] * cp[k - 1]
        R[k] = (R[k] - a[k] * R[k - 1]) / u
        cp[k] = c[k] / u
    for k in range(n - 2, -1, -1):
        R[k] -= cp[k] * R[k + 1]
    return R


def group_solve(a, b, c, r, P):
    """the kernels' split of one chunk into P parts (see the module doc)"""
    m = len(b)
    sizes = [(m + P - 1 - q) // P for q in range(P)]
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    np_ = min(P, m)                            # parts with rows
    xh, v, w = [], [], []
    for q in range(P):
        k0, mh = starts[q], sizes[q]
        if mh == 0:
            xh.append(np.zeros(0)); v.append(np.zeros(0)); w.append(np.zeros(0))
            continue
        sl = slice(k0, k0 + mh)
        R = np.zeros((mh, 3))
        R[:, 0] = r[sl]
        if q < np_ - 1:
            R[-1, 1] = c[k0 + mh - 1]         # last row -> first unknown of part q+1
        if q > 0:
            R[0, 2] = a[k0]                   # first row -> last unknown of part q-1
        X = thomas_multi(a[sl], b[sl], c[sl], R)
        xh.append(X[:, 0]); v.append(X[:, 1]); w.append(X[:, 2])

    def first(z, q):
        return z[q][0] if sizes[q] else 0.0

    def last(z, q):
        return z[q][-1] if sizes[q] else 0.0

    # unknowns L_i (x at part i's last row), R_i (x at part i+1's first row)
    N = 2 * (P - 1)
    M, rhs = np.eye(N), np.zeros(N)
    for i in range(P - 1):
        if i < np_ - 1:
            M[2 * i, 2 * i + 1] = last(v, i)
            if i > 0:
                M[2 * i, 2 * i - 2] = last(w, i)
            rhs[2 * i] = last(xh, i)
            M[2 * i + 1, 2 * i] = first(w, i + 1)
            if i + 1 < P - 1:
                M[2 * i + 1, 2 * i + 3] = first(v, i + 1)
            rhs[2 * i + 1] = first(xh, i + 1)
    z = np.linalg.solve(M, rhs)
    out = np.zeros(m)
    for q in range(P):
        if sizes[q] == 0:
            continue
        Rq = z[2 * q + 1] if q < P - 1 else 0.0
        Lq = z[2 * q - 2] if q > 0 else 0.0
        out[starts[q]:starts[q] + sizes[q]] = xh[q] - Rq * v[q] - Lq * w[q]
    return out


def eq21_like(m, rng):
    k = rng.uniform(0.05, 3.0, m)              # (B + 1/3) d^2 / dx^2
    s = rng.uniform(-0.3, 0.3, m) * k          # d d_x / (6 dx), small beside k
    a, b, c = s - k, 1.0 + 2.0 * k, -s - k
    # a wall's odd mirror folded into the first and last diagonals
    b[0] -= a[0]
    b[-1] -= c[-1]
    return a, b, c


@pytest.mark.parametrize("P", [2, 4])
def test_chunk_split_equals_direct_solve(P):
    rng = np.random.default_rng(19090415)
    for m in list(range(1, 34)) + [48, 64]:
        a, b, c = eq21_like(m, rng)
        r = rng.standard_normal(m)
        A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        x = np.linalg.solve(A, r)
        y = group_solve(a, b, c, r, P)
        assert np.max(np.abs(y - x)) <= 1e-12 * np.max(np.abs(x)), (P, m)


@pytest.mark.parametrize("P", [2, 4])
def test_chunk_split_of_a_sparse_right_hand_side(P):
    # the finalize kernel's response solve: right-hand side zero except the
    # first and the last row (the neighbour chunks' end values)
    rng = np.random.default_rng(7)
    for m in (1, 2, 3, 5, 8, 16, 31, 32):
        a, b, c = eq21_like(m, rng)
        r = np.zeros(m)
        r[0] += 0.7
        r[-1] += -1.3
        A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        x = np.linalg.solve(A, r)
        assert np.max(np.abs(group_solve(a, b, c, r, P) - x)) <= 1e-12 * np.max(np.abs(x)), (P, m)


def test_a_wrong_coupling_column_fails():
    # the construction is not vacuous: leaving the parts' coupling out (no
    # interface correction) misses the direct solution
    rng = np.random.default_rng(3)
    a, b, c = eq21_like(16, rng)
    r = rng.standard_normal(16)
    A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    x = np.linalg.solve(A, r)
    parts = np.concatenate([thomas_multi(a[:8], b[:8], c[:8], r[:8, None])[:, 0],
                            thomas_multi(a[8:], b[8:], c[8:], r[8:, None])[:, 0]])
    assert np.max(np.abs(parts - x)) > 1e-3 * np.max(np.abs(x))


def group_response(a, b, c, r0, r1, P):
    """the finalize kernel's form for a right-hand side that is r0 in the
    chunk's first row and r1 in its last: each part solves only for f and g,
    its responses to a unit value in its own first and last row, and every
    vector of the construction above is a combination of the two"""
    m = len(b)
    sizes = [(m + P - 1 - q) // P for q in range(P)]
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    np_ = min(P, m)
    f, g, aF, cL, rf, rl = [], [], [], [], [], []
    for q in range(P):
        k0, mh = starts[q], sizes[q]
        if mh == 0:
            f.append(np.zeros(0)); g.append(np.zeros(0))
            aF.append(0.0); cL.append(0.0); rf.append(0.0); rl.append(0.0)
            continue
        sl = slice(k0, k0 + mh)
        R = np.zeros((mh, 2))
        R[0, 0] = 1.0
        R[-1, 1] = 1.0
        X = thomas_multi(a[sl], b[sl], c[sl], R)
        f.append(X[:, 0]); g.append(X[:, 1])
        aF.append(a[k0] if q > 0 else 0.0)
        cL.append(c[k0 + mh - 1] if q < np_ - 1 else 0.0)
        rf.append(r0 if q == 0 else 0.0)
        rl.append(r1 if q == np_ - 1 else 0.0)

    def end(z, q, i):
        return z[q][i] if sizes[q] else 0.0

    N = 2 * (P - 1)
    M, rhs = np.eye(N), np.zeros(N)
    for i in range(P - 1):
        if i < np_ - 1:
            M[2 * i, 2 * i + 1] = cL[i] * end(g, i, -1)
            if i > 0:
                M[2 * i, 2 * i - 2] = aF[i] * end(f, i, -1)
            rhs[2 * i] = rf[i] * end(f, i, -1) + rl[i] * end(g, i, -1)
            M[2 * i + 1, 2 * i] = aF[i + 1] * end(f, i + 1, 0)
            if i + 1 < P - 1:
                M[2 * i + 1, 2 * i + 3] = cL[i + 1] * end(g, i + 1, 0)
            rhs[2 * i + 1] = rf[i + 1] * end(f, i + 1, 0) + rl[i + 1] * end(g, i + 1, 0)
    z = np.linalg.solve(M, rhs)
    out = np.zeros(m)
    for q in range(P):
        if sizes[q] == 0:
            continue
        Rq = z[2 * q + 1] if q < P - 1 else 0.0
        Lq = z[2 * q - 2] if q > 0 else 0.0
        out[starts[q]:starts[q] + sizes[q]] = (rf[q] - aF[q] * Lq) * f[q] + (rl[q] - cL[q] * Rq) * g[q]
    return out


@pytest.mark.parametrize("P", [2, 4])
def test_two_vector_response_equals_direct_solve(P):
    rng = np.random.default_rng(11)
    for m in list(range(1, 34)) + [48, 64]:
        a, b, c = eq21_like(m, rng)
        r0, r1 = rng.standard_normal(2)
        r = np.zeros(m)
        r[0] += r0
        r[-1] += r1
        A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        x = np.linalg.solve(A, r)
        y = group_response(a, b, c, r0, r1, P)
        assert np.max(np.abs(y - x)) <= 1e-12 * np.max(np.abs(x)), (P, m)
