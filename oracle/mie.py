"""Analytic sphere solutions (test infrastructure only).

* Plane-wave scattering by a sound-hard sphere of radius 1 (section 5.3):
  separation of variables with u_inc = exp(ik x.d) = sum_l i^l (2l+1)
  j_l(kr) P_l(cos t) and an outgoing scattered part sum_l a_l h_l(kr)
  P_l(cos t); the Neumann condition du/dr = 0 at r = 1 fixes
  a_l = -i^l (2l+1) j_l'(k) / h_l'(k).  With G = exp(ikr)/(4 pi r) the
  outgoing Hankel function is h_l = h_l^(1) = j_l + i y_l (the paper writes
  "second kind"; with its exp(ikr) convention only the first kind radiates).
* Pulsating sphere (section 5.2): q = 1 with the normal into the body gives
  u = 1 / (1 - ik) on the surface.
* Eigenvalues of the layer operators of eq. operator on the unit sphere for
  the Legendre densities P_l(cos t), with the normal into the body, from the
  addition theorem G = ik sum_l j_l(k r<) h_l(k r>) (2l+1)/(4 pi) P_l(cos g):
  S -> ik j_l h_l, D = M (principal value, mean of the two one-sided limits)
  -> -(ik^2/2)(j_l h_l' + j_l' h_l), H -> ik^3 j_l' h_l'.  All functions at
  argument k.
"""

from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def legendre_table(lmax: int, x: np.ndarray) -> np.ndarray:
    """P_0..P_lmax at x by the three-term recurrence; shape (lmax+1, len(x))."""
    x = np.asarray(x, dtype=np.float64)
    P = np.empty((lmax + 1,) + x.shape)
    P[0] = 1.0
    if lmax >= 1:
        P[1] = x
    for l in range(1, lmax):
        P[l + 1] = ((2 * l + 1) * x * P[l] - l * P[l - 1]) / (l + 1)
    return P


def sph_hankel1(l, z, derivative=False):
    return spherical_jn(l, z, derivative) + 1j * spherical_yn(l, z, derivative)


def default_lmax(k: float) -> int:
    return int(k + 12.0 * max(k, 1.0) ** (1.0 / 3.0) + 30)


def mie_hard_total_surface(k: float, cos_theta: np.ndarray, lmax: int | None = None) -> np.ndarray:
    """Total field u = u_inc + u_s on the unit sphere, sound-hard,
    incident exp(ik x.d); cos_theta = x.d."""
    lmax = default_lmax(k) if lmax is None else lmax
    l = np.arange(lmax + 1)
    jl = spherical_jn(l, k)
    hl = sph_hankel1(l, k)
    jlp = spherical_jn(l, k, True)
    hlp = sph_hankel1(l, k, True)
    coef = (1j ** l) * (2 * l + 1) * (jl - jlp / hlp * hl)
    P = legendre_table(lmax, cos_theta)
    return coef @ P


def mie_hard_total_field(k: float, r: np.ndarray, cos_theta: np.ndarray, lmax: int | None = None) -> np.ndarray:
    """Total field at radius r >= 1 (same series, used to check du/dr = 0)."""
    lmax = default_lmax(k * float(np.max(r))) if lmax is None else lmax
    l = np.arange(lmax + 1)[:, None]
    r = np.asarray(r, dtype=np.float64)[None, :]
    a = -(1j ** l) * (2 * l + 1) * spherical_jn(l, k, True) / sph_hankel1(l, k, True)
    terms = (1j ** l) * (2 * l + 1) * spherical_jn(l, k * r) + a * sph_hankel1(l, k * r)
    P = legendre_table(lmax, cos_theta)
    return np.sum(terms * P, axis=0)


def mie_hard_scattered(k: float, r: np.ndarray, cos_theta: np.ndarray, lmax: int | None = None) -> np.ndarray:
    """Scattered field sum_l a_l h_l(kr) P_l(cos t) at radius r >= 1."""
    lmax = default_lmax(k) if lmax is None else lmax
    l = np.arange(lmax + 1)[:, None]
    r = np.asarray(r, dtype=np.float64)[None, :]
    a = -(1j ** l) * (2 * l + 1) * spherical_jn(l, k, True) / sph_hankel1(l, k, True)
    P = legendre_table(lmax, cos_theta)
    return np.sum(a * sph_hankel1(l, k * r) * P, axis=0)


def pulsating_sphere(k: float) -> complex:
    return 1.0 / (1.0 - 1j * k)


def sphere_spectra(k: float, l: int) -> dict:
    """Eigenvalues on P_l(cos t) for the unit sphere, normal into the body."""
    j, jp = spherical_jn(l, k), spherical_jn(l, k, True)
    h, hp = sph_hankel1(l, k), sph_hankel1(l, k, True)
    S = 1j * k * j * h
    D = -(1j * k * k / 2.0) * (j * hp + jp * h)
    H = 1j * k ** 3 * jp * hp
    alpha = 1j / k
    return {"S": S, "D": D, "M": D, "H": H, "BM": 0.5 + D + alpha * H, "CBIE": 0.5 + D}
