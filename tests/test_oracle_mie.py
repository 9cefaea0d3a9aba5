"""Pins of the analytic sphere solutions (sections 5.2 and 5.3)."""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import spherical_jn

from oracle import mie


def test_wronskian():
    for k in (0.7, 5.0, 50.0):
        l = np.arange(0, int(k) + 20)
        j, jp = spherical_jn(l, k), spherical_jn(l, k, True)
        h, hp = mie.sph_hankel1(l, k), mie.sph_hankel1(l, k, True)
        assert np.allclose(j * hp - jp * h, 1j / k**2, rtol=1e-10, atol=0)


@pytest.mark.parametrize("k", [2.0, 5.0, 20.0])
def test_mie_satisfies_neumann_condition(k):
    ct = np.cos(np.linspace(0, np.pi, 13))
    h = 1e-5
    up = mie.mie_hard_total_field(k, np.full(ct.shape, 1 + h), ct)
    um = mie.mie_hard_total_field(k, np.full(ct.shape, 1 + 2 * h), ct)
    u0 = mie.mie_hard_total_field(k, np.ones_like(ct), ct)
    dudr = (-3 * u0 + 4 * up - um) / (2 * h)
    assert np.max(np.abs(dudr)) < 1e-6 * k * np.max(np.abs(u0)) * 50
    # on the surface the series equals the compact surface form
    assert np.allclose(u0, mie.mie_hard_total_surface(k, ct), rtol=1e-10, atol=1e-12)


def test_mie_paper_series_form():
    """u = u_inc + sum_m [-i^m (2m+1) j'_m/h'_m] h_m P_m on r = 1 (section 5.3)."""
    k = 5.0
    ct = np.cos(np.linspace(0, np.pi, 9))
    L = mie.default_lmax(k)
    l = np.arange(L + 1)
    coef = -(1j ** l) * (2 * l + 1) * spherical_jn(l, k, True) / mie.sph_hankel1(l, k, True) * mie.sph_hankel1(l, k)
    us = coef @ mie.legendre_table(L, ct)
    u = np.exp(1j * k * ct) + us
    assert np.allclose(u, mie.mie_hard_total_surface(k, ct), rtol=1e-12, atol=1e-12)


def test_mie_far_field_is_outgoing():
    k, ct = 3.0, np.array([0.3])
    r1, r2 = 200.0, 200.0 + np.pi / k
    us1 = mie.mie_hard_scattered(k, np.array([r1]), ct)
    us2 = mie.mie_hard_scattered(k, np.array([r2]), ct)
    # the scattered part of the full series at moderate r matches
    rr = np.array([1.7])
    assert np.allclose(mie.mie_hard_total_field(k, rr, ct) - np.exp(1j * k * rr * ct),
                       mie.mie_hard_scattered(k, rr, ct), rtol=1e-10)
    # exp(ikr)/r: half a wavelength further the value flips sign and scales r1/r2
    assert abs(us2 / us1 + r1 / r2) < 1e-2


def _single_layer_quad(k, l):
    """Apply S to P_l(cos t) at the north pole by 2-D quadrature."""
    def f(phi, t, part):
        y = np.array([np.sin(t) * np.cos(phi), np.sin(t) * np.sin(phi), np.cos(t)])
        r = np.linalg.norm(np.array([0, 0, 1.0]) - y)
        v = np.exp(1j * k * r) / (4 * np.pi * r) * mie.legendre_table(l, np.array([np.cos(t)]))[l, 0] * np.sin(t)
        return v.real if part == 0 else v.imag
    re = integrate.dblquad(lambda p, t: f(p, t, 0), 0, np.pi, 0, 2 * np.pi, epsabs=1e-11, epsrel=1e-11)[0]
    im = integrate.dblquad(lambda p, t: f(p, t, 1), 0, np.pi, 0, 2 * np.pi, epsabs=1e-11, epsrel=1e-11)[0]
    return re + 1j * im


def _double_layer_quad(k, l, r0=1.0):
    """Apply D (normal into the body, n_y = -y) at x = (0,0,r0)."""
    x = np.array([0, 0, r0])

    def f(t, part):
        # axisymmetric: integrate over phi analytically by quadrature inside
        def g(phi):
            y = np.array([np.sin(t) * np.cos(phi), np.sin(t) * np.sin(phi), np.cos(t)])
            d = x - y
            r = np.linalg.norm(d)
            G = np.exp(1j * k * r) / (4 * np.pi * r)
            return G * (1 / r - 1j * k) * (d @ (-y)) / r
        v = integrate.quad(lambda p: g(p).real, 0, 2 * np.pi, epsabs=1e-12)[0] + 1j * integrate.quad(lambda p: g(p).imag, 0, 2 * np.pi, epsabs=1e-12)[0]
        v *= mie.legendre_table(l, np.array([np.cos(t)]))[l, 0] * np.sin(t)
        return v.real if part == 0 else v.imag
    pts = [0.0, 1e-3, 1e-2, 0.1, np.pi]
    re = sum(integrate.quad(lambda t: f(t, 0), a, b, epsabs=1e-11, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))
    im = sum(integrate.quad(lambda t: f(t, 1), a, b, epsabs=1e-11, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))
    return re + 1j * im


@pytest.mark.parametrize("l", [0, 2])
def test_sphere_spectra_S_and_D_by_quadrature(l):
    k = 2.0
    sp_ = mie.sphere_spectra(k, l)
    assert abs(_single_layer_quad(k, l) - sp_["S"]) < 1e-7
    assert abs(_double_layer_quad(k, l) - sp_["D"]) < 1e-6


def test_pulsating_sphere_from_spectra():
    """Neumann data q = 1: (1/2 + D) u = (S + alpha M) q - alpha q / 2 on the
    l = 0 mode gives the closed form u = 1/(1 - ik) (section 5.2)."""
    for k in (2 * np.pi, 4 * np.pi, 3.3):
        s = mie.sphere_spectra(k, 0)
        a = 1j / k
        u = (s["S"] + a * s["M"] - 0.5 * a) / s["BM"]
        assert abs(u - mie.pulsating_sphere(k)) < 1e-12
        # CBIE alone is singular at the characteristic frequencies k = n pi
    assert abs(mie.sphere_spectra(2 * np.pi, 0)["CBIE"]) < 1e-12


# ---- the series at the wavenumbers of the large runs (section 5.3: k = 157.1
# for the paper's 4M-node sphere, k = 500 for kD = 1000) ---------------------
HIGH_K = [157.1, 500.0]


@pytest.mark.parametrize("k", HIGH_K)
def test_wronskian_over_the_whole_truncated_series(k):
    """j_l h_l' - j_l' h_l = i / k^2 for every l the surface series uses."""
    l = np.arange(0, mie.default_lmax(k) + 1)
    j, jp = spherical_jn(l, k), spherical_jn(l, k, True)
    h, hp = mie.sph_hankel1(l, k), mie.sph_hankel1(l, k, True)
    assert np.allclose(j * hp - jp * h, 1j / k**2, rtol=1e-9, atol=0)


@pytest.mark.parametrize("k", HIGH_K)
def test_neumann_condition_at_high_k(k):
    """du/dr = 0 on r = 1 by a fourth-order central difference of the full
    series (analytic in r, so it can be evaluated just inside the sphere)."""
    ct = np.cos(np.linspace(0, np.pi, 11))
    h = 2e-6
    f = {s: mie.mie_hard_total_field(k, np.full(ct.shape, 1 + s * h), ct, lmax=mie.default_lmax(k))
         for s in (-2, -1, 0, 1, 2)}
    dudr = (-f[2] + 8 * f[1] - 8 * f[-1] + f[-2]) / (12 * h)
    scale = k * np.max(np.abs(f[0]))
    assert np.max(np.abs(dudr)) < 1e-6 * scale
    # the same derivative of the incident wave alone is of order k |u|
    uinc = lambda r: np.exp(1j * k * r * ct)
    dinc = (-uinc(1 + 2 * h) + 8 * uinc(1 + h) - 8 * uinc(1 - h) + uinc(1 - 2 * h)) / (12 * h)
    assert np.max(np.abs(dinc)) > 0.5 * k
    assert np.allclose(f[0], mie.mie_hard_total_surface(k, ct), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("k", HIGH_K)
def test_series_tail_converged(k):
    """Extending the truncated series by 100 terms changes nothing, and the
    surface field equals the Wronskian form (i/k^2) sum i^l (2l+1) P_l / h_l'
    that uses h_l' alone."""
    ct = np.cos(np.linspace(0, np.pi, 201))
    L = mie.default_lmax(k)
    u = mie.mie_hard_total_surface(k, ct)
    u_more = mie.mie_hard_total_surface(k, ct, lmax=L + 100)
    assert np.max(np.abs(u - u_more)) < 1e-12 * np.max(np.abs(u))
    l = np.arange(L + 1)
    alt = (1j / k**2) * ((1j ** l) * (2 * l + 1) / mie.sph_hankel1(l, k, True)) @ mie.legendre_table(L, ct)
    assert np.allclose(u, alt, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("k", HIGH_K)
def test_geometric_optics_limit(k):
    """At ka >> 1 the illuminated pole of a rigid sphere sees the incident
    wave plus its specular reflection (reflection coefficient +1): |u| -> 2
    with O(1/k) corrections; the shadow side is far weaker than the lit side."""
    u = mie.mie_hard_total_surface(k, np.array([-1.0, -0.999, 0.5]))
    assert abs(abs(u[0]) - 2.0) < 10.0 / k
    assert abs(abs(u[1]) - 2.0) < 10.0 / k
    assert abs(u[0] / np.exp(-1j * k) - 2.0) < 10.0 / k   # phase of the incident wave at z = -1
    assert abs(u[2]) < 0.5


@pytest.mark.parametrize("k", HIGH_K)
def test_outgoing_far_field_and_optical_theorem(k):
    """Far from the sphere the scattered field radiates (du_s/dr = ik u_s to
    O(1/kr)), and energy is conserved: the extinction (4 pi / k) Im f(0)
    equals the scattered power integrated over the sphere at infinity, with
    f the far-field amplitude u_s ~ f exp(ikr)/r.  |f|^2 is a polynomial of
    degree 2 lmax in cos(theta), so Gauss-Legendre with lmax + 2 nodes
    integrates it exactly."""
    L = mie.default_lmax(k)
    R = 1e9
    x, wq = np.polynomial.legendre.leggauss(L + 2)
    us = mie.mie_hard_scattered(k, np.full(x.shape, R), x)
    f = us * R * np.exp(-1j * k * R)
    sigma_sc = 2 * np.pi * np.sum(wq * np.abs(f) ** 2)
    f0 = mie.mie_hard_scattered(k, np.array([R]), np.array([1.0]))[0] * R * np.exp(-1j * k * R)
    sigma_ext = 4 * np.pi / k * f0.imag
    assert abs(sigma_sc - sigma_ext) < 1e-6 * sigma_ext
    # geometric cross-section limit of a hard sphere: 2 pi a^2 (extinction paradox)
    assert abs(sigma_ext / (2 * np.pi) - 1.0) < 0.1
    r0 = 1e5
    d = 1e-3 / k
    ct = np.array([0.3])
    ud = (mie.mie_hard_scattered(k, np.array([r0 + d]), ct) - mie.mie_hard_scattered(k, np.array([r0 - d]), ct)) / (2 * d)
    u0 = mie.mie_hard_scattered(k, np.array([r0]), ct)
    assert abs(ud[0] / (1j * k * u0[0]) - 1.0) < 1e-3
