"""Pins of the oracle's locally corrected Nystrom operator (section 2.2)
against the analytic unit-sphere spectra of S, D, M, H (derived from the
addition theorem, cross-checked by 2-D quadrature in test_oracle_mie) and the
pulsating-sphere closed form (section 5.2).  Errors must fall with the mesh
size at the rates a quadratic-geometry Nystrom method gives."""
import numpy as np
import pytest

import synth
from oracle import mie, near, quadrature as q

OPS = {"S": (1, 0, 1, 0), "D": (0, 1, 1, 0), "M": (1, 0, 0, 1), "H": (0, 1, 0, 1)}


def _spectral_errors(n, k, l):
    el = synth.octa_sphere(n)
    pts, nrm, w = q.nystrom_nodes(el)
    ct = pts[:, 2] / np.linalg.norm(pts, axis=1)
    P = mie.legendre_table(l, ct)[l].astype(complex)
    rows = np.arange(0, len(w), max(1, len(w) // 60))
    sp = mie.sphere_spectra(k, l)
    out = {}
    for name, co in OPS.items():
        v = near.corrected_rows(el, P, k, coefs=tuple(complex(c) for c in co), rows=rows, free_term=0.0)
        out[name] = float(np.linalg.norm(v - sp[name] * P[rows]) / np.linalg.norm(sp[name] * P[rows]))
    return out


@pytest.mark.parametrize("l", [0, 2])
def test_layer_operators_converge_to_sphere_spectra(l):
    k = 2.0
    e4 = _spectral_errors(4, k, l)
    e8 = _spectral_errors(8, k, l)
    for name in ("S", "D", "H"):
        assert e8[name] < 5e-3, (name, e8)
        assert e4[name] / e8[name] > 3.0, (name, e4, e8)
    # the target-normal operator converges more slowly (normal error O(h^2))
    assert e8["M"] < 5e-2 and e4["M"] / e8["M"] > 1.5, (e4, e8)


def test_burton_miller_operators_and_pulsating_sphere():
    """BM_H = 1/2 + D + alpha H and BM_G = S + alpha M on the constant mode;
    q = 1 then gives u = (BM_G q - alpha q / 2) / BM_H -> 1/(1 - ik)."""
    k = 2 * np.pi  # a characteristic frequency of the unit sphere (section 5.2)
    el = synth.octa_sphere(8)
    n = 6 * el.shape[0]
    rows = np.arange(0, n, 61)
    one = np.ones(n, complex)
    h = near.corrected_rows(el, one, k, "H", rows=rows)
    g = near.corrected_rows(el, one, k, "G", rows=rows)
    sp = mie.sphere_spectra(k, 0)
    a = 1j / k
    assert np.max(np.abs(h - sp["BM"])) < 2e-2 * abs(sp["BM"])
    u = (g - 0.5 * a) / h
    assert np.max(np.abs(u - mie.pulsating_sphere(k))) < 3e-2 * abs(mie.pulsating_sphere(k))
    # the plain CBIE (alpha = 0) is singular here: its l = 0 eigenvalue vanishes
    assert abs(sp["CBIE"]) < 1e-12
