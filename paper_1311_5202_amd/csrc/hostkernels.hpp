// Host-side (set-up) evaluation of the Helmholtz fundamental solution and its
// normal derivatives, G = exp(ikr)/(4 pi r) with d = x - y, r = |d|
// (paper eq. fundsol and the kernels of eqs. eq_hmat, eq_gmat).
#pragma once

#include <cmath>
#include <complex>

namespace fdbem {

using cplx = std::complex<double>;

struct KVals {
    cplx G, Gny, Gnx, Gnxny;
};

// Coefficients of K = (c0 + c1 d/dn_y)(d0 + d1 d/dn_x) G.
struct OpCoef {
    cplx c0, c1, d0, d1;
};

inline KVals kernel_all(const double *x, const double *nx, const double *y, const double *ny, double k)
{
    const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const double r = std::sqrt(r2), ir = 1.0 / r;
    const double dnx = nx ? d0 * nx[0] + d1 * nx[1] + d2 * nx[2] : 0.0;
    const double dny = ny ? d0 * ny[0] + d1 * ny[1] + d2 * ny[2] : 0.0;
    const double nn = (nx && ny) ? nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2] : 0.0;
    const cplx e = std::polar(1.0, k * r);
    const cplx G = e * (ir / (4.0 * M_PI));
    const cplx a = cplx(ir, -k);  // 1/r - ik
    KVals v;
    v.G = G;
    v.Gny = G * a * (dny * ir);
    v.Gnx = -G * a * (dnx * ir);
    const cplx q = cplx(k * k - 3.0 * ir * ir, 3.0 * k * ir);  // k^2 + 3ik/r - 3/r^2
    v.Gnxny = G * (q * (dnx * dny * ir * ir) + a * (nn * ir));
    return v;
}

inline cplx kernel_combo(const double *x, const double *nx, const double *y, const double *ny, double k,
                         const OpCoef &c)
{
    KVals v = kernel_all(x, nx, y, ny, k);
    return c.c0 * c.d0 * v.G + c.c1 * c.d0 * v.Gny + c.c0 * c.d1 * v.Gnx + c.c1 * c.d1 * v.Gnxny;
}

// Single-layer value only (translation operators between equivalent points).
inline cplx kernel_G(const double *x, const double *y, double k)
{
    const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    const double r = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    return std::polar(1.0 / (4.0 * M_PI * r), k * r);
}

}  // namespace fdbem
