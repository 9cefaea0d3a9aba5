"""The product's locally corrected near-field table (host set-up through the
C ABI) against the oracle's independent element integrals: the operator
1/2 u + sum_{j != i} w_j K u_j + (correction table) u must equal the oracle's
corrected rows to the accuracy of the two quadratures."""
import numpy as np
import pytest

import oracle
import paper_1311_5202_amd as fdb
import synth
from oracle import near


@pytest.mark.parametrize("op,oop,free,tol,coupling", [("BM_H", "H", 0.5, 1e-7, 1.0), ("BM_G", "G", 0.0, 2e-6, 1.0),
                                                      ("BM_H", "H", 0.5, 1e-7, -1.0)])
def test_correction_table_matches_oracle(op, oop, free, tol, coupling):
    el = synth.octa_sphere(6)
    pts, nrm, w = fdb.nystrom_nodes(el)
    k = 4.0
    C = fdb.near_correction(el, pts, nrm, w, k, op, coupling=coupling)
    n = len(w)
    assert C.shape == (n, n)
    u = synth.random_densities(n, 5)
    rows = np.arange(0, n, 11)
    # alpha = i coupling / k in both products (eq. eq_bm)
    c0, c1, d0, _ = oracle.op_coefficients(oop, k)
    coefs = (c0, c1, d0, 1j * coupling / k)
    prod = free * u[rows] + oracle.dense_rows(pts, nrm, w, u, k, oop, rows=rows, coefs=coefs) + (C @ u)[rows]
    ref = near.corrected_rows(el, u, k, oop, rows=rows, coefs=coefs)
    assert oracle.rel_l2(prod, ref) < tol


def test_local_region_is_the_paper_rule():
    """Every stored column belongs to an element within twice its longest side
    (checked by brute-force sampling of the curved element), and the row's own
    element is always present."""
    from oracle import quadrature as q

    el = synth.octa_sphere(4)
    pts, nrm, w = fdb.nystrom_nodes(el)
    C = fdb.near_correction(el, pts, nrm, w, 3.0, "BM_H").tocsr()
    L = np.max(np.stack([np.linalg.norm(el[:, a] - el[:, (a + 1) % 3], axis=1) for a in range(3)]), axis=0)
    G = 60
    s, t = np.meshgrid(np.linspace(0, 1, G + 1), np.linspace(0, 1, G + 1))
    m = (s + t) <= 1 + 1e-12
    N, _, _ = q.shape_p2(s[m], t[m])
    Y = np.einsum("ga,ead->egd", N, el)
    for i in range(0, len(w), 29):
        d = np.min(np.linalg.norm(Y - pts[i], axis=2), axis=1)
        cols = C.indices[C.indptr[i]:C.indptr[i + 1]]
        elems = np.unique(cols // 6)
        assert i // 6 in elems
        # stored elements are within the rule (sampling can only overestimate the distance)
        assert np.all(d[elems] <= 2 * L[elems] * (1 + 2e-3))
        # clearly-inside elements are stored
        inside = np.where(d < 2 * L * (1 - 2e-2))[0]
        assert set(inside) <= set(elems)
        assert len(cols) == 6 * len(elems)
