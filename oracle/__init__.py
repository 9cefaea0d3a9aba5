"""Oracle for the fast directional Burton-Miller BEM -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 CPU implementations of what the GPU path computes:

* ``kernels`` / ``dense_rows`` / ``dense_matrix``: the Helmholtz fundamental
  solution and its normal derivatives, and the straightforward point-kernel
  summation (paper section 2, eqs. fundsol, eq_hmat, eq_gmat; section 5.1,
  eq. eq_sum) -- the exact result the fast directional algorithm reaches to
  its controlling accuracy.
* ``quadrature``: the Nystrom nodes, normals and weights (section 2.2).
* ``near``: the locally corrected near-field integrals (section 2.2, eq.
  near field / local correction) and the full Burton-Miller operator.
* ``mie``: analytic sphere solutions used to pin the solve.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the product.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import mie, quadrature  # noqa: F401
from ._lib import build, lib  # noqa: F401

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int64_p = ctypes.POINTER(ctypes.c_int64)


def _p(a):
    return a.ctypes.data_as(_c_double_p)


def op_coefficients(op: str, k: float):
    """(c0, c1, d0, d1) of K = (c0 + c1 d/dn_y)(d0 + d1 d/dn_x) G, alpha = i/k."""
    alpha = 1j / k
    table = {
        "H": (0.0, 1.0, 1.0, alpha),      # eq. eq_hmat
        "G": (1.0, 0.0, 1.0, alpha),      # eq. eq_gmat
        "T1": (1.0, alpha, 1.0, 0.0),     # eq. eq_sum (section 5.1)
        "S": (1.0, 0.0, 1.0, 0.0),
        "D": (0.0, 1.0, 1.0, 0.0),
        "M": (1.0, 0.0, 0.0, 1.0),
        "HS": (0.0, 1.0, 0.0, 1.0),
    }
    return tuple(complex(c) for c in table[op])


def _coef_array(coefs):
    return np.array([v for c in coefs for v in (c.real, c.imag)], dtype=np.float64)


def kernels(x, nx, y, ny, k):
    """(G, dG/dn_y, dG/dn_x, d2G/dn_x dn_y) at one pair."""
    out = np.zeros(8)
    f = lib().oracle_kernels
    f.restype = None
    args = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, nx, y, ny)]
    f(*[_p(a) for a in args], ctypes.c_double(k), _p(out))
    return out[0::2] + 1j * out[1::2]


def dense_rows(pts, nrm, w, u, k, op="H", rows=None, coefs=None):
    """p_i = sum_{j != i} w_j K(x_i, y_j) u_j for i in rows (all if None)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    n = len(w)
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    coefs = op_coefficients(op, k) if coefs is None else coefs
    ca = _coef_array(coefs)
    out = np.zeros(len(rows), dtype=np.complex128)
    f = lib().oracle_dense_rows
    f.restype = None
    f(ctypes.c_int64(n), _p(pts), _p(nrm), _p(w), u.ctypes.data_as(_c_double_p), ctypes.c_int64(len(rows)),
      rows.ctypes.data_as(_c_int64_p), ctypes.c_double(k), _p(ca), out.ctypes.data_as(_c_double_p))
    return out


def dense_matrix(pts, nrm, w, k, op="H", rows=None, coefs=None):
    """Rows of the point-kernel matrix w_j K(x_i, y_j), zero diagonal."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = len(w)
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    coefs = op_coefficients(op, k) if coefs is None else coefs
    ca = _coef_array(coefs)
    mat = np.zeros((len(rows), n), dtype=np.complex128)
    f = lib().oracle_dense_matrix
    f.restype = None
    f(ctypes.c_int64(n), _p(pts), _p(nrm), _p(w), ctypes.c_int64(len(rows)), rows.ctypes.data_as(_c_int64_p),
      ctypes.c_double(k), _p(ca), mat.ctypes.data_as(_c_double_p))
    return mat


def num_threads() -> int:
    f = lib().oracle_num_threads
    f.restype = ctypes.c_int
    return int(f())


def rel_l2(a, b) -> float:
    """Relative L2 error ||a - b|| / ||b|| (the error measure of section 5.1)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


from . import near  # noqa: E402,F401
