"""Oracle Nystrom discretisation (paper section 2.2) -- test infrastructure only.

The boundary is a union of curved quadratic triangles; each element carries
the six points of a degree-4 Gauss rule on the triangle, so N = 6 N_e.  The
rule is not typed in from a table: it is obtained here by solving its moment
equations (two three-point orbits (a, a, 1-2a) and (b, b, 1-2b) in
barycentric coordinates, exact for the S3-invariant polynomials 1, e2, e3,
e2^2, which makes it exact for every polynomial of degree <= 4).

Node numbering inside an element (an interface convention):
    g = 0, 1, 2 : (xi1, xi2) = (a, a), (1-2a, a), (a, 1-2a)
    g = 3, 4, 5 : (xi1, xi2) = (b, b), (1-2b, b), (b, 1-2b)
with a > b.  Global node index = 6 * element + g.

Normals point into the body (out of the acoustic domain), the orientation
under which the integral representation of section 2.1 holds with a plus
sign in front of the double-layer term.
"""

from __future__ import annotations

import numpy as np


def _moment_residual(v):
    a, b, wa, wb = v

    def e2(t):
        return 2 * t - 3 * t * t

    def e3(t):
        return t * t * (1 - 2 * t)

    return np.array([
        3 * wa + 3 * wb - 1.0 / 2.0,
        3 * wa * e2(a) + 3 * wb * e2(b) - 1.0 / 8.0,
        3 * wa * e3(a) + 3 * wb * e3(b) - 1.0 / 120.0,
        3 * wa * e2(a) ** 2 + 3 * wb * e2(b) ** 2 - 1.0 / 30.0,
    ])


def gauss6_rule():
    """Return (xi (6,2), weights (6,)) on the reference triangle of area 1/2."""
    v = np.array([0.44, 0.09, 0.11, 0.055])
    for _ in range(100):
        f = _moment_residual(v)
        J = np.empty((4, 4))
        h = 1e-7
        for c in range(4):
            dv = np.zeros(4)
            dv[c] = h
            J[:, c] = (_moment_residual(v + dv) - _moment_residual(v - dv)) / (2 * h)
        step = np.linalg.solve(J, f)
        v = v - step
        if np.max(np.abs(step)) < 1e-16:
            break
    a, b, wa, wb = v
    xi = np.array([[a, a], [1 - 2 * a, a], [a, 1 - 2 * a], [b, b], [1 - 2 * b, b], [b, 1 - 2 * b]])
    w = np.array([wa, wa, wa, wb, wb, wb])
    return xi, w


def shape_p2(xi1, xi2):
    """Quadratic Lagrange shape functions for corners 0,1,2 and mid-edges
    (0,1), (1,2), (2,0); reference corners (0,0), (1,0), (0,1)."""
    L0 = 1.0 - xi1 - xi2
    L1 = xi1
    L2 = xi2
    N = np.stack([L0 * (2 * L0 - 1), L1 * (2 * L1 - 1), L2 * (2 * L2 - 1), 4 * L0 * L1, 4 * L1 * L2, 4 * L2 * L0], -1)
    # derivatives wrt xi1 and xi2 (L0 depends on both)
    dN1 = np.stack([-(4 * L0 - 1), 4 * L1 - 1, 0 * L2, 4 * (L0 - L1), 4 * L2, -4 * L2], -1)
    dN2 = np.stack([-(4 * L0 - 1), 0 * L1, 4 * L2 - 1, -4 * L1, 4 * L1, 4 * (L0 - L2)], -1)
    return N, dN1, dN2


def element_map(elem, xi1, xi2):
    """Position, tangents y_,1 y_,2 of one element (6,3) at reference points."""
    N, d1, d2 = shape_p2(np.asarray(xi1, float), np.asarray(xi2, float))
    return N @ elem, d1 @ elem, d2 @ elem


def nystrom_nodes(elements: np.ndarray):
    """Nodes, unit normals (into the body) and weights for (Ne, 6, 3) elements.

    Returns pts (N,3), nrm (N,3), w (N,) with N = 6 Ne in the documented
    node numbering."""
    elements = np.asarray(elements, dtype=np.float64)
    xi, wq = gauss6_rule()
    N, d1, d2 = shape_p2(xi[:, 0], xi[:, 1])  # (6 pts, 6 shape)
    pos = np.einsum("ga,ead->egd", N, elements)
    t1 = np.einsum("ga,ead->egd", d1, elements)
    t2 = np.einsum("ga,ead->egd", d2, elements)
    cr = np.cross(t1, t2)
    J = np.linalg.norm(cr, axis=-1)
    nrm = -cr / J[..., None]
    w = wq[None, :] * J
    return pos.reshape(-1, 3), nrm.reshape(-1, 3), w.reshape(-1)
