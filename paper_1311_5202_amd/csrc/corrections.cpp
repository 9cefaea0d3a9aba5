// Locally corrected near-field quadrature (paper section 2.2, eqs. near field,
// local correction, kcorrection).
//
// For node x_i and every element D of its local region D_i (elements whose
// distance to x_i is at most twice their longest side) the six corrected
// weights solve  sum_g wbar_g phi_n(xi_g) = int_D K(x_i, y) phi_n dS,
// phi_n in {1, xi1, xi2, xi1^2, xi1 xi2, xi2^2}.  The mat-vec's point sum
// already holds w_j K(x_i, y_j) for every j != i, so the table stores
// dw_ij = wbar_j - [j != i] w_j K(x_i, y_j).
//
// Integrals:
//  * x_i off the element: adaptive 4-way subdivision of the reference
//    triangle until each piece is at least one diameter away from x_i, then a
//    collapsed (Duffy) tensor Gauss rule on each piece.
//  * x_i on the element (one of its Gauss points xi0): polar coordinates
//    (rho, theta) about xi0 on the three sub-triangles.  The kernels G,
//    dG/dn_y, dG/dn_x times the polar Jacobian are bounded; the
//    hypersingular d2G/dn_x dn_y is taken in the finite-part sense with a
//    spherical exclusion (Guiggiani's direct method): its Laplace part has the
//    expansion F = F_-2/rho^2 + F_-1/rho + O(1), which is subtracted and
//    integrated analytically in rho, leaving
//      FP = int int [F - F_-2/rho^2 - F_-1/rho] + int [F_-1 ln(rho_hat |A|)
//           - F_-2 (1/rho_hat - A.B/|A|^2)] dtheta,
//    with y - x = rho A + rho^2 B along the ray (exact for quadratic maps).
#include <algorithm>
#include <array>
#include <cmath>
#include <stdexcept>
#include <vector>

#include "plan.hpp"

namespace fdbem {

namespace {

// Gauss-Legendre nodes/weights on [0, 1] by Newton on P_n.
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double pp = 0;
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

struct Rule2D {
    std::vector<double> s, t, w;  // reference triangle (area 1/2)
};

// collapsed Gauss: (u, v) in [0,1]^2 -> (s, t) = (u, v (1 - u)), Jacobian (1 - u)
Rule2D duffy_rule(int n)
{
    std::vector<double> x, w;
    gauss_legendre01(n, x, w);
    Rule2D R;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            R.s.push_back(x[a]);
            R.t.push_back(x[b] * (1 - x[a]));
            R.w.push_back(w[a] * w[b] * (1 - x[a]));
        }
    return R;
}

inline void basis6(double s, double t, double phi[6])
{
    phi[0] = 1;
    phi[1] = s;
    phi[2] = t;
    phi[3] = s * s;
    phi[4] = s * t;
    phi[5] = t * t;
}

inline void basis6_grad(double s, double t, double gs[6], double gt[6])
{
    gs[0] = 0, gt[0] = 0;
    gs[1] = 1, gt[1] = 0;
    gs[2] = 0, gt[2] = 1;
    gs[3] = 2 * s, gt[3] = 0;
    gs[4] = t, gt[4] = s;
    gs[5] = 0, gt[5] = 2 * t;
}

inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// second derivatives of the quadratic map (constant over the element)
void element_second(const double *el, double y11[3], double y12[3], double y22[3])
{
    // d2N/ds2, d2N/dsdt, d2N/dt2 for corners 0,1,2 and mid-edges 01,12,20
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

struct Ctx {
    double k;
    OpCoef c;          // kernel coefficients
    Rule2D rule;       // for regular pieces
    std::vector<double> gx, gw;  // 1-D Gauss on [0,1] for polar integration
};

inline cplx kernel_at(const Ctx &C, const double *x, const double *nx, const double *y, const double *ny)
{
    return kernel_combo(x, nx, y, ny, C.k, C.c);
}

// Regular / near-singular moments over the sub-triangle with reference
// vertices v0, v1, v2 (adaptive subdivision).
void moments_regular(const Ctx &C, const double *el, const double *x, const double *nx, const double v[3][2],
                     int depth, cplx m[6])
{
    // physical size and distance estimate of the piece
    double P[3][3], yc[3], ys[3], yt[3];
    for (int a = 0; a < 3; ++a) element_eval(el, v[a][0], v[a][1], P[a], ys, yt);
    element_eval(el, (v[0][0] + v[1][0] + v[2][0]) / 3, (v[0][1] + v[1][1] + v[2][1]) / 3, yc, ys, yt);
    double diam = 0, rad = 0;
    for (int a = 0; a < 3; ++a) {
        for (int b = a + 1; b < 3; ++b) {
            const double d[3] = {P[a][0] - P[b][0], P[a][1] - P[b][1], P[a][2] - P[b][2]};
            diam = std::max(diam, std::sqrt(dot3(d, d)));
        }
        const double d[3] = {P[a][0] - yc[0], P[a][1] - yc[1], P[a][2] - yc[2]};
        rad = std::max(rad, std::sqrt(dot3(d, d)));
    }
    const double dc[3] = {x[0] - yc[0], x[1] - yc[1], x[2] - yc[2]};
    const double dist = std::sqrt(dot3(dc, dc)) - 1.2 * rad;
    if (dist < 1.0 * diam && depth < 12) {
        const double m01[2] = {0.5 * (v[0][0] + v[1][0]), 0.5 * (v[0][1] + v[1][1])};
        const double m12[2] = {0.5 * (v[1][0] + v[2][0]), 0.5 * (v[1][1] + v[2][1])};
        const double m20[2] = {0.5 * (v[2][0] + v[0][0]), 0.5 * (v[2][1] + v[0][1])};
        const double sub[4][3][2] = {{{v[0][0], v[0][1]}, {m01[0], m01[1]}, {m20[0], m20[1]}},
                                     {{m01[0], m01[1]}, {v[1][0], v[1][1]}, {m12[0], m12[1]}},
                                     {{m20[0], m20[1]}, {m12[0], m12[1]}, {v[2][0], v[2][1]}},
                                     {{m12[0], m12[1]}, {m20[0], m20[1]}, {m01[0], m01[1]}}};
        for (int q = 0; q < 4; ++q) moments_regular(C, el, x, nx, sub[q], depth + 1, m);
        return;
    }
    // affine map of the piece: xi = v0 + s (v1 - v0) + t (v2 - v0); area ratio
    const double e1[2] = {v[1][0] - v[0][0], v[1][1] - v[0][1]}, e2[2] = {v[2][0] - v[0][0], v[2][1] - v[0][1]};
    const double jac = std::fabs(e1[0] * e2[1] - e1[1] * e2[0]);
    for (size_t q = 0; q < C.rule.w.size(); ++q) {
        const double s = v[0][0] + C.rule.s[q] * e1[0] + C.rule.t[q] * e2[0];
        const double t = v[0][1] + C.rule.s[q] * e1[1] + C.rule.t[q] * e2[1];
        double y[3], a1[3], a2[3], N[3];
        element_eval(el, s, t, y, a1, a2);
        cross3(a1, a2, N);
        const double J = std::sqrt(dot3(N, N));
        const double ny[3] = {-N[0] / J, -N[1] / J, -N[2] / J};
        const cplx K = kernel_at(C, x, nx, y, ny) * (C.rule.w[q] * jac * J);
        double phi[6];
        basis6(s, t, phi);
        for (int n = 0; n < 6; ++n) m[n] += K * phi[n];
    }
}

// Singular moments with x = y(xi0) on the element.
void moments_singular(const Ctx &C, const double *el, const double xi0[2], cplx m[6])
{
    double x[3], a1[3], a2[3], N0[3];
    element_eval(el, xi0[0], xi0[1], x, a1, a2);
    cross3(a1, a2, N0);
    const double J0 = std::sqrt(dot3(N0, N0));
    const double nx[3] = {-N0[0] / J0, -N0[1] / J0, -N0[2] / J0};
    double y11[3], y12[3], y22[3];
    element_second(el, y11, y12, y22);
    const cplx hyp = C.c.c1 * C.c.d1;  // coefficient of d2G/dn_x dn_y
    const double V[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    const int nq = (int)C.gx.size();
    double phi0[6], gs[6], gt[6];
    basis6(xi0[0], xi0[1], phi0);
    basis6_grad(xi0[0], xi0[1], gs, gt);
    for (int edge = 0; edge < 3; ++edge) {
        const double *pa = V[edge], *pb = V[(edge + 1) % 3];
        const double th_a = std::atan2(pa[1] - xi0[1], pa[0] - xi0[0]);
        double th_b = std::atan2(pb[1] - xi0[1], pb[0] - xi0[0]);
        while (th_b < th_a) th_b += 2 * M_PI;
        const double dth = th_b - th_a;
        // edge line: points p = pa + u (pb - pa); ray xi0 + rho e hits it at rho_hat
        const double ex = pb[0] - pa[0], ey = pb[1] - pa[1];
        for (int qa = 0; qa < nq; ++qa) {
            const double th = th_a + dth * C.gx[qa], wth = dth * C.gw[qa];
            const double e[2] = {std::cos(th), std::sin(th)};
            // solve xi0 + rho e = pa + u (pb - pa)
            const double det = e[0] * (-ey) - e[1] * (-ex);
            const double rx = pa[0] - xi0[0], ry = pa[1] - xi0[1];
            const double rho_hat = (rx * (-ey) - ry * (-ex)) / det;
            // ray geometry: y - x = rho A + rho^2 B
            double A[3], B[3];
            for (int d = 0; d < 3; ++d) {
                A[d] = a1[d] * e[0] + a2[d] * e[1];
                B[d] = 0.5 * (y11[d] * e[0] * e[0] + 2 * y12[d] * e[0] * e[1] + y22[d] * e[1] * e[1]);
            }
            // N(rho) = N0 + rho N1 + rho^2 N2 with y_,a(rho) = a_a + rho b_a
            double b1[3], b2[3];
            for (int d = 0; d < 3; ++d) {
                b1[d] = y11[d] * e[0] + y12[d] * e[1];
                b2[d] = y12[d] * e[0] + y22[d] * e[1];
            }
            double c1[3], c2[3], N1[3];
            cross3(b1, a2, c1);
            cross3(a1, b2, c2);
            for (int d = 0; d < 3; ++d) N1[d] = c1[d] + c2[d];
            const double a2n = dot3(A, A), aa = std::sqrt(a2n);
            const double AB = dot3(A, B);
            // n_x . N with the paper's normal orientation (into the body): n_x = -N0/J0 and
            // the unit source normal n_y = -N/J, so n_x.n_y J = N0.N/J0.
            const double nN1 = dot3(N0, N1) / J0;
            // Laplace hypersingular expansion (see header):
            // F_-2 = phi0 J0 / (4 pi a^3),  F_-1 = [J0 phi1 + phi0 (nN1 - 3 J0 A.B / a^2)] / (4 pi a^3)
            const double inv4pia3 = 1.0 / (4.0 * M_PI * a2n * aa);
            double Fm2[6], Fm1[6];
            for (int n = 0; n < 6; ++n) {
                const double phi1 = gs[n] * e[0] + gt[n] * e[1];
                Fm2[n] = phi0[n] * J0 * inv4pia3;
                Fm1[n] = (J0 * phi1 + phi0[n] * (nN1 - 3.0 * J0 * AB / a2n)) * inv4pia3;
            }
            // radial integral
            for (int qr = 0; qr < nq; ++qr) {
                const double rho = rho_hat * C.gx[qr], wr = rho_hat * C.gw[qr];
                const double s = xi0[0] + rho * e[0], t = xi0[1] + rho * e[1];
                double y[3], ys[3], yt[3], N[3];
                element_eval(el, s, t, y, ys, yt);
                cross3(ys, yt, N);
                const double J = std::sqrt(dot3(N, N));
                const double ny[3] = {-N[0] / J, -N[1] / J, -N[2] / J};
                const cplx K = kernel_at(C, x, nx, y, ny) * (J * rho);
                double phi[6];
                basis6(s, t, phi);
                for (int n = 0; n < 6; ++n) {
                    cplx f = K * phi[n];
                    if (hyp != 0.0) f -= hyp * (Fm2[n] / (rho * rho) + Fm1[n] / rho);
                    m[n] += f * (wr * wth);
                }
            }
            if (hyp != 0.0)
                for (int n = 0; n < 6; ++n)
                    m[n] += hyp * (Fm1[n] * std::log(rho_hat * aa) - Fm2[n] * (1.0 / rho_hat - AB / a2n)) * wth;
        }
    }
}

// distance from x to the curved element: the smaller of an interior
// stationary point (Newton from the best grid sample) and the minima along the
// three curved edges (sampling plus Newton on the 1-D distance)
double element_distance(const double *el, const double *x)
{
    auto f_at = [&](double s, double t) {
        double y[3], a1[3], a2[3];
        element_eval(el, s, t, y, a1, a2);
        const double d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
        return dot3(d, d);
    };
    double best = 1e300, bs = 1.0 / 3, bt = 1.0 / 3;
    const int G = 12;
    for (int i = 0; i <= G; ++i)
        for (int j = 0; i + j <= G; ++j) {
            const double f = f_at((double)i / G, (double)j / G);
            if (f < best) best = f, bs = (double)i / G, bt = (double)j / G;
        }
    // interior Newton (Gauss-Newton on |y - x|^2)
    {
        double s = bs, t = bt;
        for (int it = 0; it < 30; ++it) {
            double y[3], a1[3], a2[3];
            element_eval(el, s, t, y, a1, a2);
            const double d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
            const double g1 = dot3(a1, d), g2 = dot3(a2, d);
            const double h11 = dot3(a1, a1), h12 = dot3(a1, a2), h22 = dot3(a2, a2);
            const double det = h11 * h22 - h12 * h12;
            if (det <= 0) break;
            const double ds = -(h22 * g1 - h12 * g2) / det, dt = -(-h12 * g1 + h11 * g2) / det;
            s += ds;
            t += dt;
            if (s < -0.5 || t < -0.5 || s + t > 1.5) break;
            if (std::fabs(ds) + std::fabs(dt) < 1e-15) break;
        }
        if (s >= 0 && t >= 0 && s + t <= 1) best = std::min(best, f_at(s, t));
    }
    // edges: (u,0), (1-u,u), (0,1-u)
    for (int e = 0; e < 3; ++e) {
        auto pt = [&](double u, double &s, double &t) {
            if (e == 0) s = u, t = 0;
            else if (e == 1) s = 1 - u, t = u;
            else s = 0, t = 1 - u;
        };
        const int M = 32;
        double bu = 0, bf = 1e300;
        for (int q = 0; q <= M; ++q) {
            double s, t;
            pt((double)q / M, s, t);
            const double f = f_at(s, t);
            if (f < bf) bf = f, bu = (double)q / M;
        }
        // golden-section refinement on the bracketing interval
        double a = std::max(0.0, bu - 1.0 / M), b = std::min(1.0, bu + 1.0 / M);
        const double gr = 0.5 * (std::sqrt(5.0) - 1);
        for (int it = 0; it < 80; ++it) {
            const double c1 = b - gr * (b - a), c2 = a + gr * (b - a);
            double s1, t1, s2, t2;
            pt(c1, s1, t1);
            pt(c2, s2, t2);
            if (f_at(s1, t1) < f_at(s2, t2)) b = c2; else a = c1;
        }
        double s, t;
        pt(0.5 * (a + b), s, t);
        bf = std::min(bf, f_at(s, t));
        best = std::min(best, bf);
    }
    return std::sqrt(best);
}

double element_longest_side(const double *el)
{
    double L = 0;
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3;
        const double d[3] = {el[3 * a] - el[3 * b], el[3 * a + 1] - el[3 * b + 1], el[3 * a + 2] - el[3 * b + 2]};
        L = std::max(L, std::sqrt(dot3(d, d)));
    }
    return L;
}

// inverse transpose of the 6x6 basis matrix V_gn = phi_n(xi_g)
std::array<double, 36> vandermonde_inv_t()
{
    double xi[6][2], wq[6];
    gauss6(xi, wq);
    double M[6][12];
    for (int n = 0; n < 6; ++n) {
        for (int g = 0; g < 6; ++g) {
            double phi[6];
            basis6(xi[g][0], xi[g][1], phi);
            M[n][g] = phi[n];  // V^T(n, g)
        }
        for (int c = 0; c < 6; ++c) M[n][6 + c] = (n == c);
    }
    for (int c = 0; c < 6; ++c) {
        int p = c;
        for (int r = c + 1; r < 6; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[p][c])) p = r;
        for (int q = 0; q < 12; ++q) std::swap(M[c][q], M[p][q]);
        const double d = M[c][c];
        for (int q = 0; q < 12; ++q) M[c][q] /= d;
        for (int r = 0; r < 6; ++r)
            if (r != c) {
                const double f = M[r][c];
                for (int q = 0; q < 12; ++q) M[r][q] -= f * M[c][q];
            }
    }
    std::array<double, 36> out;  // out[g*6+n] = (V^T)^-1 (g, n)
    for (int g = 0; g < 6; ++g)
        for (int n = 0; n < 6; ++n) out[g * 6 + n] = M[g][6 + n];
    return out;
}

}  // namespace

// Builds the correction table of one operator (coefficients c) in caller order.
static void build_table(Plan &P, const OpCoef &c, std::vector<int64_t> &rp, std::vector<int64_t> &col,
                        std::vector<cplx> &val)
{
    const int64_t ne = P.n_elem, N = P.N;
    // caller-order node data
    std::vector<double> X(3 * N), NX(3 * N), W(N);
    for (int64_t s = 0; s < N; ++s) {
        const int64_t i = P.perm[s];
        X[3 * i] = P.px[s];
        X[3 * i + 1] = P.py[s];
        X[3 * i + 2] = P.pz[s];
        NX[3 * i] = P.pnx[s];
        NX[3 * i + 1] = P.pny[s];
        NX[3 * i + 2] = P.pnz[s];
        W[i] = P.pw[s];
    }
    // element centres, radii, longest sides; uniform grid over centres
    std::vector<double> ec(3 * ne), er(ne), eL(ne);
    double rmax = 0;
    for (int64_t e = 0; e < ne; ++e) {
        const double *el = &P.elem[18 * e];
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
        eL[e] = element_longest_side(el);
        rmax = std::max(rmax, 2 * eL[e] + er[e]);
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t e = 0; e < ne; ++e)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], ec[3 * e + d]);
            hi[d] = std::max(hi[d], ec[3 * e + d]);
        }
    const double cell = std::max(rmax, 1e-12);
    int dims[3];
    for (int d = 0; d < 3; ++d) dims[d] = std::max(1, (int)std::ceil((hi[d] - lo[d]) / cell) + 1);
    const int64_t ncell = (int64_t)dims[0] * dims[1] * dims[2];
    std::vector<int64_t> cstart(ncell + 1, 0), cidx(ne);
    auto cell_of = [&](const double *p, int ijk[3]) {
        for (int d = 0; d < 3; ++d) ijk[d] = std::min(dims[d] - 1, std::max(0, (int)std::floor((p[d] - lo[d]) / cell)));
    };
    std::vector<int64_t> ecell(ne);
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
    Ctx C;
    C.k = P.k;
    C.c = c;
    C.rule = duffy_rule(8);
    gauss_legendre01(32, C.gx, C.gw);
    const std::array<double, 36> Vit = vandermonde_inv_t();
    double xi[6][2], wq[6];
    gauss6(xi, wq);
    // per-row lists, then CSR
    std::vector<std::vector<std::pair<int64_t, cplx>>> rows(N);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        const double *x = &X[3 * i], *nx = &NX[3 * i];
        int ijk[3];
        cell_of(x, ijk);
        auto &row = rows[i];
        for (int a = std::max(0, ijk[0] - 1); a <= std::min(dims[0] - 1, ijk[0] + 1); ++a)
            for (int b = std::max(0, ijk[1] - 1); b <= std::min(dims[1] - 1, ijk[1] + 1); ++b)
                for (int d = std::max(0, ijk[2] - 1); d <= std::min(dims[2] - 1, ijk[2] + 1); ++d) {
                    const int64_t q = ((int64_t)a * dims[1] + b) * dims[2] + d;
                    for (int64_t t = cstart[q]; t < cstart[q + 1]; ++t) {
                        const int64_t e = cidx[t];
                        const double dc[3] = {x[0] - ec[3 * e], x[1] - ec[3 * e + 1], x[2] - ec[3 * e + 2]};
                        if (std::sqrt(dot3(dc, dc)) > 2 * eL[e] + er[e]) continue;
                        const double *el = &P.elem[18 * e];
                        const bool self = (i / 6 == e);
                        if (!self && element_distance(el, x) > 2 * eL[e]) continue;
                        cplx m[6] = {0, 0, 0, 0, 0, 0};
                        if (self) {
                            moments_singular(C, el, xi[i % 6], m);
                        } else {
                            const double v[3][2] = {{0, 0}, {1, 0}, {0, 1}};
                            moments_regular(C, el, x, nx, v, 0, m);
                        }
                        for (int g = 0; g < 6; ++g) {
                            cplx wb = 0;
                            for (int n = 0; n < 6; ++n) wb += Vit[g * 6 + n] * m[n];
                            const int64_t j = 6 * e + g;
                            if (j != i) wb -= W[j] * kernel_combo(x, nx, &X[3 * j], &NX[3 * j], P.k, c);
                            row.push_back({j, wb});
                        }
                    }
                }
        std::sort(row.begin(), row.end(), [](const auto &p, const auto &q) { return p.first < q.first; });
    }
    rp.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) rp[i + 1] = rp[i] + (int64_t)rows[i].size();
    col.resize(rp[N]);
    val.resize(rp[N]);
    for (int64_t i = 0; i < N; ++i) {
        int64_t p = rp[i];
        for (auto &pr : rows[i]) {
            col[p] = pr.first;
            val[p] = pr.second;
            ++p;
        }
    }
}

void correction_table_host(int64_t n_elem, const double *elem, const double *pts, const double *nrm, const double *w,
                           double k, int op, std::vector<int64_t> &rp, std::vector<int64_t> &col,
                           std::vector<cplx> &val)
{
    Plan P;
    P.N = 6 * n_elem;
    P.k = k;
    P.n_elem = n_elem;
    P.elem.assign(elem, elem + 18 * n_elem);
    P.perm.resize(P.N);
    P.px.resize(P.N), P.py.resize(P.N), P.pz.resize(P.N), P.pnx.resize(P.N), P.pny.resize(P.N), P.pnz.resize(P.N);
    P.pw.assign(w, w + P.N);
    for (int64_t i = 0; i < P.N; ++i) {
        P.perm[i] = i;
        P.px[i] = pts[3 * i], P.py[i] = pts[3 * i + 1], P.pz[i] = pts[3 * i + 2];
        P.pnx[i] = nrm[3 * i], P.pny[i] = nrm[3 * i + 1], P.pnz[i] = nrm[3 * i + 2];
    }
    const cplx al(0.0, 1.0 / k);
    const OpCoef c = (op == 3) ? OpCoef{0.0, 1.0, 1.0, al} : OpCoef{1.0, 0.0, 1.0, al};
    build_table(P, c, rp, col, val);
}

void build_corrections(Plan &P)
{
    if (P.n_elem <= 0) return;
    const cplx al(0.0, 1.0 / P.k);
    if (P.opt.corrections & 1) {
        build_table(P, OpCoef{0.0, 1.0, 1.0, al}, P.corr_ptr, P.corr_col, P.corr_val);
        P.has_corr = true;
    }
    if (P.opt.corrections & 2) {
        build_table(P, OpCoef{1.0, 0.0, 1.0, al}, P.corrg_ptr, P.corrg_col, P.corrg_val);
        P.has_corr_g = true;
    }
}

}  // namespace fdbem
