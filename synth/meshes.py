"""Curved quadratic triangle meshes of closed surfaces and seeded densities.

Element layout: ``elem[e, a, :]`` with ``a`` = 0,1,2 the corner nodes and
3,4,5 the mid-edge nodes of edges (0,1), (1,2), (2,0).  Corners are ordered
counter-clockwise when the surface is seen from outside (the acoustic side),
so ``(p1 - p0) x (p2 - p0)`` points away from the body.

The sphere mesh splits each face of an octahedron into n x n flat triangles
and projects every corner and mid-edge node radially onto the surface, which
gives 8 n^2 elements and 48 n^2 Nystrom nodes (six per element): n = 8 gives
3072, n = 64 gives 196,608, n = 289 gives 4,009,008.
"""

from __future__ import annotations

import math

import numpy as np


def _octa_faces():
    faces = []
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                a = np.array([sx, 0.0, 0.0])
                b = np.array([0.0, sy, 0.0])
                c = np.array([0.0, 0.0, sz])
                if sx * sy * sz < 0:
                    b, c = c, b
                faces.append((a, b, c))
    return faces


def _flat_split(n: int) -> np.ndarray:
    """Flat subdivision of the octahedron: (8 n^2, 6, 3) points on its faces."""
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    up = (ii + jj) <= n - 1
    dn = (ii + jj) <= n - 2
    iu, ju = ii[up], jj[up]
    idn, jdn = ii[dn], jj[dn]
    # barycentric-like (i, j) grid coordinates of the three corners
    c_up = [(iu, ju), (iu + 1, ju), (iu, ju + 1)]
    c_dn = [(idn + 1, jdn), (idn + 1, jdn + 1), (idn, jdn + 1)]
    out = []
    for a, b, c in _octa_faces():
        def P(i, j):
            return a[None, :] + (i[:, None] / n) * (b - a)[None, :] + (j[:, None] / n) * (c - a)[None, :]

        for corners in (c_up, c_dn):
            p0, p1, p2 = (P(i, j) for i, j in corners)
            out.append(np.stack([p0, p1, p2, 0.5 * (p0 + p1), 0.5 * (p1 + p2), 0.5 * (p2 + p0)], axis=1))
    return np.concatenate(out, axis=0)


def octa_sphere(n: int, radius: float = 1.0) -> np.ndarray:
    """Unit (or given radius) sphere: octahedron split n x n per face, nodes
    projected radially.  Returns float64 array (8 n^2, 6, 3)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    flat = _flat_split(n)
    r = np.linalg.norm(flat, axis=-1, keepdims=True)
    return np.ascontiguousarray(radius * flat / r)


def n_for_dofs(n_dofs: float) -> int:
    """Split count n whose sphere mesh has about ``n_dofs`` = 48 n^2 nodes."""
    return max(1, int(round(math.sqrt(n_dofs / 48.0))))


def ellipsoid(n: int, aspect: float) -> np.ndarray:
    """Prolate ellipsoid with axes 1:1:aspect (sphere mesh scaled in z)."""
    s = octa_sphere(n)
    s = s.copy()
    s[..., 2] *= aspect
    return s


def _real_sph_harm(lmax: int, theta: np.ndarray, phi: np.ndarray) -> list:
    """Real spherical harmonics up to degree lmax (unnormalised associated
    Legendre times cos/sin), enough to build smooth random radial bumps."""
    from scipy.special import lpmv

    x = np.cos(theta)
    out = []
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            p = lpmv(m, l, x) / max(1.0, math.factorial(l + m) ** 0.5)
            out.append(p * np.cos(m * phi))
            if m > 0:
                out.append(p * np.sin(m * phi))
    return out


def star_surface(n: int, seed: int, lmax: int = 4, amp: float = 0.2) -> np.ndarray:
    """Star-shaped surface r(theta, phi) = 1 + amp * S / max|S| with S a sum of
    real spherical harmonics of degree <= lmax with N(0,1) coefficients."""
    rng = np.random.default_rng(seed)
    s = octa_sphere(n)
    theta = np.arccos(np.clip(s[..., 2], -1.0, 1.0))
    phi = np.arctan2(s[..., 1], s[..., 0])
    basis = _real_sph_harm(lmax, theta, phi)
    coef = rng.standard_normal(len(basis))
    S = sum(c * b for c, b in zip(coef, basis))
    # normalise by the max over a fine sample of the sphere, not only the nodes
    tt, pp = np.meshgrid(np.linspace(0, math.pi, 181), np.linspace(-math.pi, math.pi, 361))
    Sf = sum(c * b for c, b in zip(coef, _real_sph_harm(lmax, tt, pp)))
    r = 1.0 + amp * S / np.max(np.abs(Sf))
    return np.ascontiguousarray(s * r[..., None])


def random_densities(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex densities with real and imaginary parts i.i.d. U[-1, 1]."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, n)
    im = rng.uniform(-1.0, 1.0, n)
    return (re + 1j * im).astype(dtype)


def random_directions(count: int, seed: int) -> np.ndarray:
    """Unit vectors uniform on the sphere."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def instance_batch(count: int, seed: int, n_range=(10_000, 100_000), kd_range=(5.0, 60.0)):
    """Seeded list of (elements, k, kind) for uneven-size batches: spheres,
    prolate ellipsoids (axis ratio U[1,4]) and star-shaped surfaces, node
    count U[n_range], kD U[kd_range] with D the largest extent."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = int(rng.integers(0, 3))
        n = n_for_dofs(rng.uniform(*n_range))
        kd = rng.uniform(*kd_range)
        if kind == 0:
            el = octa_sphere(n)
            name = "sphere"
        elif kind == 1:
            el = ellipsoid(n, rng.uniform(1.0, 4.0))
            name = "ellipsoid"
        else:
            el = star_surface(n, int(rng.integers(0, 2**31 - 1)))
            name = "star"
        pts = el.reshape(-1, 3)
        D = float(np.max(pts.max(0) - pts.min(0)))
        out.append((el, kd / D, name))
    return out
