"""Pins of the oracle's kernels and dense sums against things other than
themselves: symbolic differentiation of G = exp(ikr)/(4 pi r) (eq. fundsol),
finite differences, reciprocity, the Laplace limit and the Helmholtz
equation (eq. helmholtz)."""
import numpy as np
import pytest
import sympy as sp


def _sympy_kernels():
    x = sp.symbols("x0:3", real=True)
    y = sp.symbols("y0:3", real=True)
    nx = sp.symbols("nx0:3", real=True)
    ny = sp.symbols("ny0:3", real=True)
    k = sp.symbols("k", positive=True)
    r = sp.sqrt(sum((x[i] - y[i]) ** 2 for i in range(3)))
    G = sp.exp(sp.I * k * r) / (4 * sp.pi * r)
    Gny = sum(ny[i] * sp.diff(G, y[i]) for i in range(3))
    Gnx = sum(nx[i] * sp.diff(G, x[i]) for i in range(3))
    Gxy = sum(nx[i] * sp.diff(Gny, x[i]) for i in range(3))
    args = (*x, *nx, *y, *ny, k)
    return [sp.lambdify(args, e, "mpmath") for e in (G, Gny, Gnx, Gxy)]


def _rand_pair(rng, dist):
    x = rng.standard_normal(3)
    d = rng.standard_normal(3)
    d *= dist / np.linalg.norm(d)
    nx = rng.standard_normal(3); nx /= np.linalg.norm(nx)
    ny = rng.standard_normal(3); ny /= np.linalg.norm(ny)
    return x, nx, x - d, ny


def test_kernels_match_symbolic_derivatives(oracle_lib):
    import mpmath
    mpmath.mp.dps = 30
    fs = _sympy_kernels()
    rng = np.random.default_rng(11)
    for dist in (1e-3, 0.07, 0.9, 13.0):
        for k in (0.3, 5.0, 157.1):
            x, nx, y, ny = _rand_pair(rng, dist)
            got = oracle_lib.kernels(x, nx, y, ny, k)
            args = [mpmath.mpf(float(v)) for v in (*x, *nx, *y, *ny)] + [mpmath.mpf(k)]
            for g, f in zip(got, fs):
                ref = complex(f(*args))
                assert abs(g - ref) <= 1e-12 * abs(ref) + 1e-300, (dist, k, g, ref)


def test_kernels_finite_differences(oracle_lib):
    rng = np.random.default_rng(3)
    k, h = 4.0, 1e-5
    x, nx, y, ny = _rand_pair(rng, 0.8)
    K = oracle_lib.kernels(x, nx, y, ny, k)
    Gp = oracle_lib.kernels(x, nx, y + h * ny, ny, k)[0]
    Gm = oracle_lib.kernels(x, nx, y - h * ny, ny, k)[0]
    assert abs((Gp - Gm) / (2 * h) - K[1]) < 1e-8 * abs(K[1])
    Gp = oracle_lib.kernels(x + h * nx, nx, y, ny, k)[0]
    Gm = oracle_lib.kernels(x - h * nx, nx, y, ny, k)[0]
    assert abs((Gp - Gm) / (2 * h) - K[2]) < 1e-8 * abs(K[2])
    Fp = oracle_lib.kernels(x + h * nx, nx, y, ny, k)[1]
    Fm = oracle_lib.kernels(x - h * nx, nx, y, ny, k)[1]
    assert abs((Fp - Fm) / (2 * h) - K[3]) < 1e-7 * abs(K[3])


def test_helmholtz_equation_and_laplace_limit(oracle_lib):
    rng = np.random.default_rng(5)
    k, h = 3.0, 1e-3
    x, nx, y, ny = _rand_pair(rng, 1.3)
    G0 = oracle_lib.kernels(x, nx, y, ny, k)[0]
    lap = 0
    for d in range(3):
        e = np.zeros(3); e[d] = h
        lap += oracle_lib.kernels(x + e, nx, y, ny, k)[0] + oracle_lib.kernels(x - e, nx, y, ny, k)[0] - 2 * G0
    lap /= h * h
    assert abs(lap + k * k * G0) < 1e-5 * abs(k * k * G0)
    # k -> 0: d2G/dnx dny -> (nx.ny - 3 (d.nx)(d.ny)/r^2) / (4 pi r^3)
    d = x - y
    r = np.linalg.norm(d)
    lapl = (nx @ ny - 3 * (d @ nx) * (d @ ny) / r**2) / (4 * np.pi * r**3)
    assert abs(oracle_lib.kernels(x, nx, y, ny, 1e-7)[3] - lapl) < 1e-9 * abs(lapl)


def test_reciprocity(oracle_lib):
    rng = np.random.default_rng(9)
    for _ in range(5):
        x, nx, y, ny = _rand_pair(rng, 0.5)
        a = oracle_lib.kernels(x, nx, y, ny, 7.0)
        b = oracle_lib.kernels(y, ny, x, nx, 7.0)
        assert abs(a[0] - b[0]) < 1e-14 * abs(a[0])
        assert abs(a[1] - b[2]) < 1e-13 * abs(a[1])   # dG/dn_y(x,y) = dG/dn_x(y,x)
        assert abs(a[3] - b[3]) < 1e-13 * abs(a[3])


def test_dense_sum_indexing_against_sympy_sum(oracle_lib):
    """Tiny brute-force sum with the symbolically differentiated kernels."""
    import mpmath
    fs = _sympy_kernels()
    rng = np.random.default_rng(1)
    n, k = 9, 2.5
    pts = rng.standard_normal((n, 3))
    nrm = rng.standard_normal((n, 3)); nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    w = rng.uniform(0.5, 1.5, n)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for op, (c0, c1, d0, d1) in (("H", (0, 1, 1, 1j / k)), ("G", (1, 0, 1, 1j / k)), ("T1", (1, 1j / k, 1, 0))):
        got = oracle_lib.dense_rows(pts, nrm, w, u, k, op)
        for i in range(n):
            acc = 0
            for j in range(n):
                if j == i:
                    continue
                args = [mpmath.mpf(float(v)) for v in (*pts[i], *nrm[i], *pts[j], *nrm[j])] + [mpmath.mpf(k)]
                G, Gy, Gx, Gxy = (complex(f(*args)) for f in fs)
                acc += w[j] * (c0 * d0 * G + c1 * d0 * Gy + c0 * d1 * Gx + c1 * d1 * Gxy) * u[j]
            assert abs(got[i] - acc) < 1e-12 * max(1, abs(acc)), (op, i)


def test_bilinear_reciprocity_between_calls(oracle_lib):
    """a^T (D u) = u^T (M a) with unit weights (D_ij = M_ji)."""
    rng = np.random.default_rng(2)
    n, k = 300, 6.0
    pts = rng.standard_normal((n, 3))
    nrm = rng.standard_normal((n, 3)); nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    w = np.ones(n)
    a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Du = oracle_lib.dense_rows(pts, nrm, w, u, k, "D")
    Ma = oracle_lib.dense_rows(pts, nrm, w, a, k, "M")
    assert abs(a @ Du - u @ Ma) < 1e-11 * abs(a @ Du)
    Hu = oracle_lib.dense_rows(pts, nrm, w, u, k, "HS")
    Ha = oracle_lib.dense_rows(pts, nrm, w, a, k, "HS")
    assert abs(a @ Hu - u @ Ha) < 1e-11 * abs(a @ Hu)


def test_dense_matrix_structure(oracle_lib):
    """dense_matrix against the kernel identities rather than itself: weights
    sit on the columns (source side), the diagonal is zero, the H kernel is
    symmetric under exchange of the two points with their normals, and the
    G-kernel matrix is the transpose of the Table-1 kernel matrix (since
    dG/dn_x(x,y) = dG/dn_y(y,x)), as the double-layer matrix is of the
    adjoint one, while the hypersingular kernel alone is symmetric; its
    product with u reproduces the independently accumulated dense_rows."""
    rng = np.random.default_rng(21)
    n, k = 40, 3.5
    pts = rng.standard_normal((n, 3))
    nrm = rng.standard_normal((n, 3)); nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    w = rng.uniform(0.2, 2.0, n)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    H = oracle_lib.dense_matrix(pts, nrm, w, k, "H")
    G = oracle_lib.dense_matrix(pts, nrm, w, k, "G")
    T1 = oracle_lib.dense_matrix(pts, nrm, w, k, "T1")
    assert np.all(np.diag(H) == 0) and np.all(np.diag(G) == 0)
    Khs = oracle_lib.dense_matrix(pts, nrm, w, k, "HS") / w[None, :]
    assert np.allclose(Khs, Khs.T, rtol=1e-12, atol=0)
    D = oracle_lib.dense_matrix(pts, nrm, w, k, "D") / w[None, :]
    M = oracle_lib.dense_matrix(pts, nrm, w, k, "M") / w[None, :]
    assert np.allclose(D, M.T, rtol=1e-12, atol=0)
    assert np.allclose(H / w[None, :], D + 1j / k * Khs, rtol=1e-12, atol=0)
    assert np.allclose(G / w[None, :], (T1 / w[None, :]).T, rtol=1e-12, atol=0)
    # one entry against the symbolic kernels (row/column orientation)
    import mpmath
    fs = _sympy_kernels()
    i, j = 3, 17
    args = [mpmath.mpf(float(v)) for v in (*pts[i], *nrm[i], *pts[j], *nrm[j])] + [mpmath.mpf(k)]
    Gv, Gy, Gx, Gxy = (complex(f(*args)) for f in fs)
    assert abs(H[i, j] - w[j] * (Gy + 1j / k * Gxy)) < 1e-12 * abs(H[i, j])
    assert abs(G[i, j] - w[j] * (Gv + 1j / k * Gx)) < 1e-12 * abs(G[i, j])
    for op, M in (("H", H), ("G", G), ("T1", T1)):
        rows = oracle_lib.dense_rows(pts, nrm, w, u, k, op)
        assert np.allclose(M @ u, rows, rtol=1e-12, atol=1e-14)
    sub = np.array([5, 0, 39])
    assert np.array_equal(oracle_lib.dense_matrix(pts, nrm, w, k, "H", rows=sub), H[sub])
