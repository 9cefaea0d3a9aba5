// Locally corrected near-field quadrature (paper section 2.2, eqs. near field,
// local correction, kcorrection), built on the GPU.
//
// For node x_i and every element D of its local region D_i (elements whose
// distance to x_i is at most twice their longest side) the six corrected
// weights solve  sum_g wbar_g phi_n(xi_g) = int_D K(x_i, y) phi_n dS,
// phi_n in {1, xi1, xi2, xi1^2, xi1 xi2, xi2^2}.  The mat-vec's point sum
// already holds w_j K(x_i, y_j) for every j != i, so the table stores
// dw_ij = wbar_j - [j != i] w_j K(x_i, y_j), in blocks of six (one element).
//
// Integrals:
//  * x_i off the element: adaptive 4-way subdivision of the reference
//    triangle until each piece is at least one diameter away from x_i, then an
//    8 x 8 collapsed (Duffy) Gauss rule on each piece.
//  * x_i on the element (one of its Gauss points xi0): polar coordinates
//    (rho, theta) about xi0 on the three sub-triangles, 32 x 32 Gauss points.
//    G, dG/dn_y, dG/dn_x times the polar Jacobian are bounded; the
//    hypersingular d2G/dn_x dn_y is taken in the finite-part sense with a
//    spherical exclusion (Guiggiani's direct method): its Laplace part has the
//    expansion F = F_-2/rho^2 + F_-1/rho + O(1), which is subtracted and
//    integrated analytically in rho, leaving
//      FP = int int [F - F_-2/rho^2 - F_-1/rho] + int [F_-1 ln(rho_hat |A|)
//           - F_-2 (1/rho_hat - A.B/|A|^2)] dtheta,
//    with y - x = rho A + rho^2 B along the ray (exact for quadratic maps).
//
// The same __host__ __device__ routines serve the GPU build (one thread per
// candidate (node, element) pair) and the host table of bem_near_correction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <stdexcept>
#include <string>
#include <vector>

#include "device.hpp"

namespace fdbem {

#define HIP_CHECK(expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            throw std::runtime_error(std::string("HIP error ") + hipGetErrorString(e_) + " at " + \
                                     __FILE__ + ":" + std::to_string(__LINE__));                 \
    } while (0)

namespace nq {

constexpr int NG = 32;      // 1-D Gauss points of the singular polar rule
constexpr int ND = 8;       // 1-D points of the collapsed rule on regular pieces
constexpr int STACK = 64;   // pending pieces of the adaptive subdivision

struct Tables {
    double gx[NG], gw[NG];              // Gauss-Legendre on [0, 1]
    double ds[ND * ND], dt[ND * ND], dw[ND * ND];  // collapsed rule on the reference triangle
    double xi[6][2];                    // the element's Gauss points (node numbering)
    double vinvt[36];                   // (V^T)^-1, V_gn = phi_n(xi_g)
};

struct Z {
    double x, y;
};
__host__ __device__ inline Z zadd(Z a, Z b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline Z zsub(Z a, Z b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline Z zmul(Z a, Z b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline Z zs(Z a, double s) { return {a.x * s, a.y * s}; }

struct Coef {
    Z c0, c1, d0, d1;
};

__host__ __device__ inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__host__ __device__ inline void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// (c0 + c1 d/dn_y)(d0 + d1 d/dn_x) G at x <- y, G = exp(ikr)/(4 pi r), d = x - y
__host__ __device__ inline Z kernel(const double *x, const double *nx, const double *y, const double *ny, double k,
                                    const Coef &c)
{
    const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2), ir = 1.0 / r;
    const double dnx = (d0 * nx[0] + d1 * nx[1] + d2 * nx[2]) * ir;
    const double dny = (d0 * ny[0] + d1 * ny[1] + d2 * ny[2]) * ir;
    const double nn = nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2];
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const Z G = {cs * ir * 0.07957747154594767, sn * ir * 0.07957747154594767};
    const Z a = {ir, -k};
    const Z q = {k * k - 3.0 * ir * ir, 3.0 * k * ir};
    Z t = zmul(zmul(c.c0, c.d0), Z{1.0, 0.0});
    t = zadd(t, zmul(zmul(c.c1, c.d0), zs(a, dny)));
    t = zadd(t, zmul(zmul(c.c0, c.d1), zs(a, -dnx)));
    t = zadd(t, zmul(zmul(c.c1, c.d1), zadd(zs(q, dnx * dny), zs(a, nn * ir))));
    return zmul(G, t);
}

__host__ __device__ inline void elem_eval(const double *el, double s, double t, double y[3], double ys[3],
                                          double yt[3])
{
    const double L0 = 1.0 - s - t;
    const double N[6] = {L0 * (2 * L0 - 1), s * (2 * s - 1), t * (2 * t - 1), 4 * L0 * s, 4 * s * t, 4 * t * L0};
    const double Ns[6] = {1 - 4 * L0, 4 * s - 1, 0, 4 * (L0 - s), 4 * t, -4 * t};
    const double Nt[6] = {1 - 4 * L0, 0, 4 * t - 1, -4 * s, 4 * s, 4 * (L0 - t)};
    for (int d = 0; d < 3; ++d) {
        y[d] = ys[d] = yt[d] = 0;
        for (int a = 0; a < 6; ++a) {
            y[d] += N[a] * el[3 * a + d];
            ys[d] += Ns[a] * el[3 * a + d];
            yt[d] += Nt[a] * el[3 * a + d];
        }
    }
}

__host__ __device__ inline void elem_second(const double *el, double y11[3], double y12[3], double y22[3])
{
    const double a11[6] = {4, 4, 0, -8, 0, 0};
    const double a12[6] = {4, 0, 0, -4, 4, -4};
    const double a22[6] = {4, 0, 4, 0, 0, -8};
    for (int d = 0; d < 3; ++d) {
        y11[d] = y12[d] = y22[d] = 0;
        for (int a = 0; a < 6; ++a) {
            y11[d] += a11[a] * el[3 * a + d];
            y12[d] += a12[a] * el[3 * a + d];
            y22[d] += a22[a] * el[3 * a + d];
        }
    }
}

__host__ __device__ inline void basis6(double s, double t, double p[6])
{
    p[0] = 1, p[1] = s, p[2] = t, p[3] = s * s, p[4] = s * t, p[5] = t * t;
}

__host__ __device__ inline double dist2_at(const double *el, const double *x, double s, double t)
{
    double y[3], a1[3], a2[3];
    elem_eval(el, s, t, y, a1, a2);
    const double d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
    return dot3(d, d);
}

__host__ __device__ inline void edge_point(int e, double u, double &s, double &t)
{
    if (e == 0) s = u, t = 0;
    else if (e == 1) s = 1 - u, t = u;
    else s = 0, t = 1 - u;
}

// distance from x to the curved element: the smaller of an interior stationary
// point (Gauss-Newton from the best grid sample) and the minima along the
// three curved edges (sampling plus golden-section search)
__host__ __device__ inline double elem_distance(const double *el, const double *x)
{
    double best = 1e300, bs = 1.0 / 3, bt = 1.0 / 3;
    const int G = 12;
    for (int i = 0; i <= G; ++i)
        for (int j = 0; i + j <= G; ++j) {
            const double f = dist2_at(el, x, (double)i / G, (double)j / G);
            if (f < best) best = f, bs = (double)i / G, bt = (double)j / G;
        }
    {
        double s = bs, t = bt;
        for (int it = 0; it < 30; ++it) {
            double y[3], a1[3], a2[3];
            elem_eval(el, s, t, y, a1, a2);
            const double d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
            const double g1 = dot3(a1, d), g2 = dot3(a2, d);
            const double h11 = dot3(a1, a1), h12 = dot3(a1, a2), h22 = dot3(a2, a2);
            const double det = h11 * h22 - h12 * h12;
            if (det <= 0) break;
            const double ds = -(h22 * g1 - h12 * g2) / det, dt = -(-h12 * g1 + h11 * g2) / det;
            s += ds;
            t += dt;
            if (s < -0.5 || t < -0.5 || s + t > 1.5) break;
            if (fabs(ds) + fabs(dt) < 1e-15) break;
        }
        if (s >= 0 && t >= 0 && s + t <= 1) best = fmin(best, dist2_at(el, x, s, t));
    }
    for (int e = 0; e < 3; ++e) {
        const int M = 32;
        double bu = 0, bf = 1e300;
        for (int q = 0; q <= M; ++q) {
            double s, t;
            edge_point(e, (double)q / M, s, t);
            const double f = dist2_at(el, x, s, t);
            if (f < bf) bf = f, bu = (double)q / M;
        }
        double a = fmax(0.0, bu - 1.0 / M), b = fmin(1.0, bu + 1.0 / M);
        const double gr = 0.6180339887498949;
        for (int it = 0; it < 80; ++it) {
            const double c1 = b - gr * (b - a), c2 = a + gr * (b - a);
            double s1, t1, s2, t2;
            edge_point(e, c1, s1, t1);
            edge_point(e, c2, s2, t2);
            if (dist2_at(el, x, s1, t1) < dist2_at(el, x, s2, t2)) b = c2;
            else a = c1;
        }
        double s, t;
        edge_point(e, 0.5 * (a + b), s, t);
        best = fmin(best, fmin(bf, dist2_at(el, x, s, t)));
    }
    return sqrt(best);
}

__host__ __device__ inline double longest_side(const double *el)
{
    double L = 0;
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3;
        const double d[3] = {el[3 * a] - el[3 * b], el[3 * a + 1] - el[3 * b + 1], el[3 * a + 2] - el[3 * b + 2]};
        L = fmax(L, sqrt(dot3(d, d)));
    }
    return L;
}

struct Piece {
    double v[3][2];
    int depth;
};

// moments int_D K(x, y) phi_n dS for x off the element (adaptive subdivision)
__host__ __device__ inline void moments_regular(const Tables &T, const double *el, const double *x, const double *nx,
                                                double k, const Coef &c, Z m[6])
{
    Piece stack[STACK];
    int sp = 0;
    stack[sp++] = Piece{{{0, 0}, {1, 0}, {0, 1}}, 0};
    while (sp > 0) {
        const Piece pc = stack[--sp];
        double P[3][3], yc[3], ys[3], yt[3];
        for (int a = 0; a < 3; ++a) elem_eval(el, pc.v[a][0], pc.v[a][1], P[a], ys, yt);
        elem_eval(el, (pc.v[0][0] + pc.v[1][0] + pc.v[2][0]) / 3, (pc.v[0][1] + pc.v[1][1] + pc.v[2][1]) / 3, yc, ys,
                  yt);
        double diam = 0, rad = 0;
        for (int a = 0; a < 3; ++a) {
            for (int b = a + 1; b < 3; ++b) {
                const double d[3] = {P[a][0] - P[b][0], P[a][1] - P[b][1], P[a][2] - P[b][2]};
                diam = fmax(diam, sqrt(dot3(d, d)));
            }
            const double d[3] = {P[a][0] - yc[0], P[a][1] - yc[1], P[a][2] - yc[2]};
            rad = fmax(rad, sqrt(dot3(d, d)));
        }
        const double dc[3] = {x[0] - yc[0], x[1] - yc[1], x[2] - yc[2]};
        const double dist = sqrt(dot3(dc, dc)) - 1.2 * rad;
        if (dist < diam && pc.depth < 12 && sp + 4 <= STACK) {
            const double m01[2] = {0.5 * (pc.v[0][0] + pc.v[1][0]), 0.5 * (pc.v[0][1] + pc.v[1][1])};
            const double m12[2] = {0.5 * (pc.v[1][0] + pc.v[2][0]), 0.5 * (pc.v[1][1] + pc.v[2][1])};
            const double m20[2] = {0.5 * (pc.v[2][0] + pc.v[0][0]), 0.5 * (pc.v[2][1] + pc.v[0][1])};
            const int d1 = pc.depth + 1;
            stack[sp++] = Piece{{{pc.v[0][0], pc.v[0][1]}, {m01[0], m01[1]}, {m20[0], m20[1]}}, d1};
            stack[sp++] = Piece{{{m01[0], m01[1]}, {pc.v[1][0], pc.v[1][1]}, {m12[0], m12[1]}}, d1};
            stack[sp++] = Piece{{{m20[0], m20[1]}, {m12[0], m12[1]}, {pc.v[2][0], pc.v[2][1]}}, d1};
            stack[sp++] = Piece{{{m12[0], m12[1]}, {m20[0], m20[1]}, {m01[0], m01[1]}}, d1};
            continue;
        }
        const double e1[2] = {pc.v[1][0] - pc.v[0][0], pc.v[1][1] - pc.v[0][1]};
        const double e2[2] = {pc.v[2][0] - pc.v[0][0], pc.v[2][1] - pc.v[0][1]};
        const double jac = fabs(e1[0] * e2[1] - e1[1] * e2[0]);
        for (int q = 0; q < ND * ND; ++q) {
            const double s = pc.v[0][0] + T.ds[q] * e1[0] + T.dt[q] * e2[0];
            const double t = pc.v[0][1] + T.ds[q] * e1[1] + T.dt[q] * e2[1];
            double y[3], a1[3], a2[3], N[3];
            elem_eval(el, s, t, y, a1, a2);
            cross3(a1, a2, N);
            const double J = sqrt(dot3(N, N));
            const double ny[3] = {-N[0] / J, -N[1] / J, -N[2] / J};
            const Z K = zs(kernel(x, nx, y, ny, k, c), T.dw[q] * jac * J);
            double phi[6];
            basis6(s, t, phi);
            for (int n = 0; n < 6; ++n) m[n] = zadd(m[n], zs(K, phi[n]));
        }
    }
}

// moments with x = y(xi0) on the element (finite part for d2G/dn_x dn_y)
__host__ __device__ inline void moments_singular(const Tables &T, const double *el, double s0, double t0, double k,
                                                 const Coef &c, Z m[6])
{
    double x[3], a1[3], a2[3], N0[3];
    elem_eval(el, s0, t0, x, a1, a2);
    cross3(a1, a2, N0);
    const double J0 = sqrt(dot3(N0, N0));
    const double nx[3] = {-N0[0] / J0, -N0[1] / J0, -N0[2] / J0};
    double y11[3], y12[3], y22[3];
    elem_second(el, y11, y12, y22);
    const Z hyp = zmul(c.c1, c.d1);
    const bool has_hyp = hyp.x != 0.0 || hyp.y != 0.0;
    const double V[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    double phi0[6];
    basis6(s0, t0, phi0);
    const double gs[6] = {0, 1, 0, 2 * s0, t0, 0}, gt[6] = {0, 0, 1, 0, s0, 2 * t0};
    for (int edge = 0; edge < 3; ++edge) {
        const double *pa = V[edge], *pb = V[(edge + 1) % 3];
        const double th_a = atan2(pa[1] - t0, pa[0] - s0);
        double th_b = atan2(pb[1] - t0, pb[0] - s0);
        while (th_b < th_a) th_b += 2 * M_PI;
        const double dth = th_b - th_a;
        const double ex = pb[0] - pa[0], ey = pb[1] - pa[1];
        for (int qa = 0; qa < NG; ++qa) {
            const double th = th_a + dth * T.gx[qa], wth = dth * T.gw[qa];
            const double e[2] = {cos(th), sin(th)};
            const double det = e[0] * (-ey) - e[1] * (-ex);
            const double rx = pa[0] - s0, ry = pa[1] - t0;
            const double rho_hat = (rx * (-ey) - ry * (-ex)) / det;
            double A[3], B[3], b1[3], b2[3], c1[3], c2[3], N1[3];
            for (int d = 0; d < 3; ++d) {
                A[d] = a1[d] * e[0] + a2[d] * e[1];
                B[d] = 0.5 * (y11[d] * e[0] * e[0] + 2 * y12[d] * e[0] * e[1] + y22[d] * e[1] * e[1]);
                b1[d] = y11[d] * e[0] + y12[d] * e[1];
                b2[d] = y12[d] * e[0] + y22[d] * e[1];
            }
            cross3(b1, a2, c1);
            cross3(a1, b2, c2);
            for (int d = 0; d < 3; ++d) N1[d] = c1[d] + c2[d];
            const double a2n = dot3(A, A), aa = sqrt(a2n), AB = dot3(A, B);
            // normals into the body: n_x . n_y J = N0 . N / J0
            const double nN1 = dot3(N0, N1) / J0;
            const double inv4pia3 = 1.0 / (4.0 * M_PI * a2n * aa);
            double Fm2[6], Fm1[6];
            for (int n = 0; n < 6; ++n) {
                const double phi1 = gs[n] * e[0] + gt[n] * e[1];
                Fm2[n] = phi0[n] * J0 * inv4pia3;
                Fm1[n] = (J0 * phi1 + phi0[n] * (nN1 - 3.0 * J0 * AB / a2n)) * inv4pia3;
            }
            for (int qr = 0; qr < NG; ++qr) {
                const double rho = rho_hat * T.gx[qr], wr = rho_hat * T.gw[qr];
                const double s = s0 + rho * e[0], t = t0 + rho * e[1];
                double y[3], ys[3], yt[3], N[3];
                elem_eval(el, s, t, y, ys, yt);
                cross3(ys, yt, N);
                const double J = sqrt(dot3(N, N));
                const double ny[3] = {-N[0] / J, -N[1] / J, -N[2] / J};
                const Z K = zs(kernel(x, nx, y, ny, k, c), J * rho);
                double phi[6];
                basis6(s, t, phi);
                for (int n = 0; n < 6; ++n) {
                    Z f = zs(K, phi[n]);
                    if (has_hyp) f = zsub(f, zs(hyp, Fm2[n] / (rho * rho) + Fm1[n] / rho));
                    m[n] = zadd(m[n], zs(f, wr * wth));
                }
            }
            if (has_hyp)
                for (int n = 0; n < 6; ++n)
                    m[n] = zadd(m[n], zs(hyp, (Fm1[n] * log(rho_hat * aa) - Fm2[n] * (1.0 / rho_hat - AB / a2n)) * wth));
        }
    }
}

// six table entries of one (node, element) pair
__host__ __device__ inline void pair_weights(const Tables &T, const double *el, int64_t e, int64_t i, const double *x,
                                             const double *nx, const double *X, const double *NX, const double *W,
                                             double k, const Coef &c, Z out[6])
{
    Z m[6];
    for (int n = 0; n < 6; ++n) m[n] = Z{0.0, 0.0};
    if (i / 6 == e)
        moments_singular(T, el, T.xi[i % 6][0], T.xi[i % 6][1], k, c, m);
    else
        moments_regular(T, el, x, nx, k, c, m);
    for (int g = 0; g < 6; ++g) {
        Z wb = {0.0, 0.0};
        for (int n = 0; n < 6; ++n) wb = zadd(wb, zs(m[n], T.vinvt[g * 6 + n]));
        const int64_t j = 6 * e + g;
        if (j != i) wb = zsub(wb, zs(kernel(x, nx, X + 3 * j, NX + 3 * j, k, c), W[j]));
        out[g] = wb;
    }
}

void gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 1;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1, p1 = z;
            for (int l = 2; l <= n; ++l) {
                const double p2 = ((2 * l - 1) * z * p1 - (l - 1) * p0) / l;
                p0 = p1;
                p1 = p2;
            }
            pp = n * (z * p1 - p0) / (z * z - 1);
            const double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = 0.5 * (1 - z);
        w[i] = 1.0 / ((1 - z * z) * pp * pp);
    }
}

Tables make_tables()
{
    Tables T;
    gauss_legendre01(NG, T.gx, T.gw);
    double x[ND], w[ND];
    gauss_legendre01(ND, x, w);
    for (int a = 0; a < ND; ++a)
        for (int b = 0; b < ND; ++b) {
            T.ds[a * ND + b] = x[a];
            T.dt[a * ND + b] = x[b] * (1 - x[a]);
            T.dw[a * ND + b] = w[a] * w[b] * (1 - x[a]);
        }
    double wq[6];
    gauss6(T.xi, wq);
    // (V^T)^-1 by Gauss-Jordan on V^T(n, g) = phi_n(xi_g)
    double M[6][12];
    for (int n = 0; n < 6; ++n) {
        for (int g = 0; g < 6; ++g) {
            double phi[6];
            basis6(T.xi[g][0], T.xi[g][1], phi);
            M[n][g] = phi[n];
        }
        for (int q = 0; q < 6; ++q) M[n][6 + q] = (n == q);
    }
    for (int col = 0; col < 6; ++col) {
        int p = col;
        for (int r = col + 1; r < 6; ++r)
            if (std::fabs(M[r][col]) > std::fabs(M[p][col])) p = r;
        for (int q = 0; q < 12; ++q) std::swap(M[col][q], M[p][q]);
        const double d = M[col][col];
        for (int q = 0; q < 12; ++q) M[col][q] /= d;
        for (int r = 0; r < 6; ++r)
            if (r != col) {
                const double f = M[r][col];
                for (int q = 0; q < 12; ++q) M[r][q] -= f * M[col][q];
            }
    }
    for (int g = 0; g < 6; ++g)
        for (int n = 0; n < 6; ++n) T.vinvt[g * 6 + n] = M[g][6 + n];
    return T;
}

// coefficients of K = (c0 + c1 d/dn_y)(d0 + d1 d/dn_x) G with alpha = i / ka
Coef op_coef(int op, double ka)
{
    const Z al = {0.0, 1.0 / ka}, one = {1.0, 0.0}, zero = {0.0, 0.0};
    return op == 3 ? Coef{zero, one, one, al} : Coef{one, zero, one, al};
}

// candidate (node, element) pairs: centre within 2 L + radius of the node
struct Candidates {
    std::vector<int64_t> ptr;   // per node (caller order)
    std::vector<int32_t> elem;  // element of each candidate
    std::vector<double> L;      // longest side per element
};

Candidates candidates(int64_t ne, const double *elem, const double *X)
{
    const int64_t N = 6 * ne;
    Candidates C;
    std::vector<double> ec(3 * ne), er(ne);
    C.L.resize(ne);
    double reach = 0;
    for (int64_t e = 0; e < ne; ++e) {
        const double *el = elem + 18 * e;
        double c3[3] = {0, 0, 0};
        for (int a = 0; a < 6; ++a)
            for (int d = 0; d < 3; ++d) c3[d] += el[3 * a + d] / 6;
        double r = 0;
        for (int a = 0; a < 6; ++a) {
            const double d[3] = {el[3 * a] - c3[0], el[3 * a + 1] - c3[1], el[3 * a + 2] - c3[2]};
            r = std::max(r, std::sqrt(dot3(d, d)));
        }
        for (int d = 0; d < 3; ++d) ec[3 * e + d] = c3[d];
        er[e] = 1.1 * r;  // curved sides bulge slightly past the node hull
        C.L[e] = longest_side(el);
        reach = std::max(reach, 2 * C.L[e] + er[e]);
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t e = 0; e < ne; ++e)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], ec[3 * e + d]);
            hi[d] = std::max(hi[d], ec[3 * e + d]);
        }
    const double cell = std::max(reach, 1e-12);
    int dims[3];
    for (int d = 0; d < 3; ++d) dims[d] = std::max(1, (int)std::ceil((hi[d] - lo[d]) / cell) + 1);
    const int64_t ncell = (int64_t)dims[0] * dims[1] * dims[2];
    auto cell_of = [&](const double *p, int ijk[3]) {
        for (int d = 0; d < 3; ++d) ijk[d] = std::min(dims[d] - 1, std::max(0, (int)std::floor((p[d] - lo[d]) / cell)));
    };
    std::vector<int64_t> cstart(ncell + 1, 0), cidx(ne), ecell(ne);
    for (int64_t e = 0; e < ne; ++e) {
        int ijk[3];
        cell_of(&ec[3 * e], ijk);
        ecell[e] = ((int64_t)ijk[0] * dims[1] + ijk[1]) * dims[2] + ijk[2];
        cstart[ecell[e] + 1]++;
    }
    for (int64_t q = 0; q < ncell; ++q) cstart[q + 1] += cstart[q];
    {
        std::vector<int64_t> pos(cstart.begin(), cstart.end() - 1);
        for (int64_t e = 0; e < ne; ++e) cidx[pos[ecell[e]]++] = e;
    }
    std::vector<std::vector<int32_t>> per(N);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) {
        const double *x = X + 3 * i;
        int ijk[3];
        cell_of(x, ijk);
        auto &v = per[i];
        for (int a = std::max(0, ijk[0] - 1); a <= std::min(dims[0] - 1, ijk[0] + 1); ++a)
            for (int b = std::max(0, ijk[1] - 1); b <= std::min(dims[1] - 1, ijk[1] + 1); ++b)
                for (int d = std::max(0, ijk[2] - 1); d <= std::min(dims[2] - 1, ijk[2] + 1); ++d) {
                    const int64_t q = ((int64_t)a * dims[1] + b) * dims[2] + d;
                    for (int64_t t = cstart[q]; t < cstart[q + 1]; ++t) {
                        const int64_t e = cidx[t];
                        const double dc[3] = {x[0] - ec[3 * e], x[1] - ec[3 * e + 1], x[2] - ec[3 * e + 2]};
                        if (e == i / 6 || std::sqrt(dot3(dc, dc)) <= 2 * C.L[e] + er[e]) v.push_back((int32_t)e);
                    }
                }
        std::sort(v.begin(), v.end());
    }
    C.ptr.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) C.ptr[i + 1] = C.ptr[i] + (int64_t)per[i].size();
    C.elem.resize(C.ptr[N]);
    for (int64_t i = 0; i < N; ++i) std::copy(per[i].begin(), per[i].end(), C.elem.begin() + C.ptr[i]);
    return C;
}

// ---- device kernels
__global__ void k_corr_flag(int64_t n, const int64_t *__restrict__ cnode, const int32_t *__restrict__ celem,
                            const double *__restrict__ elem, const double *__restrict__ L,
                            const double *__restrict__ X, unsigned char *__restrict__ keep)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = cnode[p];
    const int64_t e = celem[p];
    keep[p] = (i / 6 == e) || elem_distance(elem + 18 * e, X + 3 * i) <= 2.0 * L[e];
}

__global__ __launch_bounds__(128) void k_corr_weights(int64_t n, const int64_t *__restrict__ cnode,
                                                      const int32_t *__restrict__ celem,
                                                      const double *__restrict__ elem, const double *__restrict__ X,
                                                      const double *__restrict__ NX, const double *__restrict__ W,
                                                      const Tables *__restrict__ T, double k, Coef c,
                                                      double2 *__restrict__ val)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = cnode[p];
    const int64_t e = celem[p];
    Z out[6];
    pair_weights(*T, elem + 18 * e, e, i, X + 3 * i, NX + 3 * i, X, NX, W, k, c, out);
    for (int g = 0; g < 6; ++g) val[6 * p + g] = make_double2(out[g].x, out[g].y);
}

}  // namespace nq

// Host table (expanded CSR) for bem_near_correction.
void correction_table_host(int64_t n_elem, const double *elem, const double *pts, const double *nrm, const double *w,
                           double k, int op, double coupling, std::vector<int64_t> &rp, std::vector<int64_t> &col,
                           std::vector<cplx> &val)
{
    using namespace nq;
    const int64_t N = 6 * n_elem;
    const Tables T = make_tables();
    const Coef c = op_coef(op, k / coupling);
    Candidates C = candidates(n_elem, elem, pts);
    std::vector<unsigned char> keep(C.elem.size());
    std::vector<Z> v6(6 * C.elem.size());
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t p = C.ptr[i]; p < C.ptr[i + 1]; ++p) {
            const int64_t e = C.elem[p];
            keep[p] = (i / 6 == e) || elem_distance(elem + 18 * e, pts + 3 * i) <= 2.0 * C.L[e];
            if (keep[p]) pair_weights(T, elem + 18 * e, e, i, pts + 3 * i, nrm + 3 * i, pts, nrm, w, k, c, &v6[6 * p]);
        }
    rp.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) {
        int64_t cnt = 0;
        for (int64_t p = C.ptr[i]; p < C.ptr[i + 1]; ++p) cnt += keep[p] ? 6 : 0;
        rp[i + 1] = rp[i] + cnt;
    }
    col.resize(rp[N]);
    val.resize(rp[N]);
    for (int64_t i = 0; i < N; ++i) {
        int64_t q = rp[i];
        for (int64_t p = C.ptr[i]; p < C.ptr[i + 1]; ++p)
            if (keep[p])
                for (int g = 0; g < 6; ++g) {
                    col[q] = 6 * (int64_t)C.elem[p] + g;
                    val[q] = cplx(v6[6 * p + g].x, v6[6 * p + g].y);
                    ++q;
                }
    }
}

// GPU build of the block tables of the plan's operators (caller order);
// fills the device block-CSR arrays of D.
void build_corrections_device(Plan &P, Device &D)
{
    using namespace nq;
    const int64_t ne = P.n_elem, N = P.N;
    std::vector<double> X(3 * N), NX(3 * N), W(N);
    for (int64_t s = 0; s < N; ++s) {
        const int64_t i = P.perm[s];
        X[3 * i] = P.px[s], X[3 * i + 1] = P.py[s], X[3 * i + 2] = P.pz[s];
        NX[3 * i] = P.pnx[s], NX[3 * i + 1] = P.pny[s], NX[3 * i + 2] = P.pnz[s];
        W[i] = P.pw[s];
    }
    Candidates C = candidates(ne, P.elem.data(), X.data());
    const int64_t nc = (int64_t)C.elem.size();
    std::vector<int64_t> cnode(nc);
    for (int64_t i = 0; i < N; ++i)
        for (int64_t p = C.ptr[i]; p < C.ptr[i + 1]; ++p) cnode[p] = i;
    // temporary device buffers
    std::vector<void *> tmp;
    auto up = [&](const void *h, size_t bytes) {
        void *d = nullptr;
        HIP_CHECK(hipMalloc(&d, std::max<size_t>(bytes, 16)));
        tmp.push_back(d);
        if (bytes && h) HIP_CHECK(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice));
        return d;
    };
    try {
        double *dX = (double *)up(X.data(), 8 * X.size());
        double *dNX = (double *)up(NX.data(), 8 * NX.size());
        double *dW = (double *)up(W.data(), 8 * W.size());
        double *dE = (double *)up(P.elem.data(), 8 * P.elem.size());
        double *dL = (double *)up(C.L.data(), 8 * C.L.size());
        const Tables T = make_tables();
        Tables *dT = (Tables *)up(&T, sizeof(Tables));
        int64_t *dcn = (int64_t *)up(cnode.data(), 8 * (size_t)nc);
        int32_t *dce = (int32_t *)up(C.elem.data(), 4 * (size_t)nc);
        unsigned char *dkeep = (unsigned char *)up(nullptr, (size_t)nc);
        hipLaunchKernelGGL(k_corr_flag, dim3((unsigned)((nc + 127) / 128)), dim3(128), 0, 0, nc, dcn, dce, dE, dL, dX,
                           dkeep);
        HIP_CHECK(hipGetLastError());
        std::vector<unsigned char> keep(nc);
        HIP_CHECK(hipMemcpy(keep.data(), dkeep, (size_t)nc, hipMemcpyDeviceToHost));
        // compact: kept pairs, node-major
        std::vector<int64_t> rp(N + 1, 0), kn;
        std::vector<int32_t> ke;
        kn.reserve(nc);
        ke.reserve(nc);
        for (int64_t i = 0; i < N; ++i) {
            for (int64_t p = C.ptr[i]; p < C.ptr[i + 1]; ++p)
                if (keep[p]) {
                    kn.push_back(i);
                    ke.push_back(C.elem[p]);
                }
            rp[i + 1] = (int64_t)ke.size();
        }
        const int64_t nk = (int64_t)ke.size();
        int64_t *dkn = (int64_t *)up(kn.data(), 8 * (size_t)nk);
        int32_t *dke_tmp = (int32_t *)up(ke.data(), 4 * (size_t)nk);
        for (int t = 0; t < 2; ++t) {
            const int op = t == 0 ? 3 : 4;
            if (!((P.opt.corrections >> t) & 1)) continue;
            double2 *dval = nullptr;
            HIP_CHECK(hipMalloc(&dval, sizeof(double2) * 6 * (size_t)std::max<int64_t>(nk, 1)));
            D.allocs.push_back(dval);
            D.bytes += sizeof(double2) * 6 * (size_t)nk;
            const Coef c = op_coef(op, P.opt.alpha_k(P.k));
            // launch in slices so no single dispatch runs for long
            const int64_t slice = 1 << 20;
            for (int64_t b = 0; b < nk; b += slice) {
                const int64_t m = std::min(slice, nk - b);
                hipLaunchKernelGGL(k_corr_weights, dim3((unsigned)((m + 127) / 128)), dim3(128), 0, 0, m, dkn + b,
                                   dke_tmp + b, dE, dX, dNX, dW, dT, P.k, c, dval + 6 * b);
                HIP_CHECK(hipGetLastError());
            }
            HIP_CHECK(hipDeviceSynchronize());
            DCorr &Q = (t == 0) ? D.corr : D.corrg;
            Q.n_blocks = nk;
            Q.val = dval;
        }
        // shared block structure of both tables
        if (P.opt.corrections & 3) {
            int64_t *drp = nullptr;
            int32_t *dbe = nullptr;
            HIP_CHECK(hipMalloc(&drp, 8 * (N + 1)));
            HIP_CHECK(hipMalloc(&dbe, 4 * (size_t)std::max<int64_t>(nk, 1)));
            D.allocs.push_back(drp);
            D.allocs.push_back(dbe);
            D.bytes += 8 * (N + 1) + 4 * (size_t)nk;
            HIP_CHECK(hipMemcpy(drp, rp.data(), 8 * (N + 1), hipMemcpyHostToDevice));
            HIP_CHECK(hipMemcpy(dbe, ke.data(), 4 * (size_t)nk, hipMemcpyHostToDevice));
            D.corr.rp = D.corrg.rp = drp;
            D.corr.blk = D.corrg.blk = dbe;
        }
        P.has_corr = (P.opt.corrections & 1) != 0;
        P.has_corr_g = (P.opt.corrections & 2) != 0;
        P.corr_blocks = nk;
    } catch (...) {
        for (void *p : tmp) (void)hipFree(p);
        throw;
    }
    for (void *p : tmp) (void)hipFree(p);
}

}  // namespace fdbem
