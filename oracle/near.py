"""Locally corrected Nystrom operator (section 2.2) -- test infrastructure only.

``corrected_rows`` evaluates rows of  c u + sum_far w_j K u_j + sum_{D in D_i}
int_D K ut_D dS  with the oracle's own nodes, Gauss points and element
integrals (see oracle_near.c)."""

from __future__ import annotations

import ctypes

import numpy as np

from . import _lib, op_coefficients, _coef_array
from .quadrature import gauss6_rule, nystrom_nodes


def corrected_rows(elements, u, k, op="H", rows=None, free_term=None, rel_tol=1e-10, coefs=None):
    """Rows of the corrected operator.  op "H": (1/2) u + Hbar u (the sound-hard
    Burton-Miller operator, free term 1/2); op "G": Gbar q (no free term)."""
    el = np.ascontiguousarray(elements, dtype=np.float64).reshape(-1, 6, 3)
    pts, nrm, w = nystrom_nodes(el)
    xi, _ = gauss6_rule()
    n = len(w)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    if free_term is None:
        free_term = 0.5 if op == "H" else 0.0
    coefs = op_coefficients(op, k) if coefs is None else coefs
    ca = _coef_array(coefs)
    out = np.zeros(len(rows), dtype=np.complex128)
    dp = ctypes.POINTER(ctypes.c_double)
    f = _lib.lib().oracle_corrected_rows
    f.restype = None
    g = np.ascontiguousarray(xi, dtype=np.float64)
    f(ctypes.c_int64(el.shape[0]), el.ctypes.data_as(dp), pts.ctypes.data_as(dp), nrm.ctypes.data_as(dp),
      w.ctypes.data_as(dp), g.ctypes.data_as(dp), u.ctypes.data_as(dp), ctypes.c_int64(len(rows)),
      rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.c_double(k), ca.ctypes.data_as(dp),
      ctypes.c_double(free_term), ctypes.c_double(rel_tol), out.ctypes.data_as(dp))
    return out

