"""Pins of the oracle's Nystrom discretisation (section 2.2): exactness of the
derived six-point rule, flat-element integrals, sphere area convergence and
the normal orientation fixed by the integral representation (section 2.1)."""
import math

import numpy as np

from oracle import quadrature as q
import synth


def test_rule_exact_to_degree_4_and_not_5():
    xi, w = q.gauss6_rule()
    assert abs(w.sum() - 0.5) < 1e-15
    worst5 = 0.0
    for p in range(7):
        for r in range(7 - p):
            exact = math.factorial(p) * math.factorial(r) / math.factorial(p + r + 2)
            val = float(np.sum(w * xi[:, 0] ** p * xi[:, 1] ** r))
            if p + r <= 4:
                assert abs(val - exact) < 2e-15, (p, r)
            elif p + r == 5:
                worst5 = max(worst5, abs(val - exact))
    assert worst5 > 1e-6
    # all points strictly inside, positive weights
    assert np.all(xi > 0) and np.all(xi.sum(1) < 1) and np.all(w > 0)


def test_flat_element_polynomials():
    rng = np.random.default_rng(0)
    v = rng.standard_normal((3, 3))
    el = np.vstack([v, 0.5 * (v[0] + v[1]), 0.5 * (v[1] + v[2]), 0.5 * (v[2] + v[0])])[None]
    pts, nrm, w = q.nystrom_nodes(el)
    area = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    assert abs(w.sum() - area) < 1e-13 * area
    # integral of x^2 over the triangle: exact via edge-midpoint rule for quadratics
    mids = [0.5 * (v[0] + v[1]), 0.5 * (v[1] + v[2]), 0.5 * (v[2] + v[0])]
    exact = area / 3 * sum(m[0] ** 2 for m in mids)
    assert abs(np.sum(w * pts[:, 0] ** 2) - exact) < 1e-12 * max(1, abs(exact))


def test_sphere_area_converges_and_normals_point_inward():
    errs = []
    for n in (2, 4, 8):
        pts, nrm, w = q.nystrom_nodes(synth.octa_sphere(n))
        errs.append(abs(w.sum() - 4 * math.pi))
        r = np.linalg.norm(pts, axis=1)
        # normals: unit and into the body (opposite to the radial direction)
        assert np.allclose(np.linalg.norm(nrm, axis=1), 1, atol=1e-14)
        assert np.all(np.sum(nrm * pts / r[:, None], axis=1) < -0.98)
    # quadratic geometry: area error drops at least ~8x per halving of h
    assert errs[1] < errs[0] / 8 and errs[2] < errs[1] / 8
