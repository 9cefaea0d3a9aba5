/*
 * Oracle for the locally corrected Nystrom operator -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64 CPU code, slow on purpose, sharing nothing with the product.
 *
 * Row i of the operator applied to nodal values u (paper section 2.2, eqs.
 * ndbie, far field, near field, local correction, kcorrection):
 *
 *   (A u)_i = c u_i + sum_{D not in D_i} sum_{j in D} w_j K(x_i, y_j) u_j
 *                   + sum_{D in D_i} int_D K(x_i, y) ut_D(y) dS_y
 *
 * where D_i holds the elements whose distance to x_i is at most twice their
 * longest side, and ut_D is the polynomial in span{xi1^p xi2^q, p+q <= 2}
 * taking the nodal values at the element's six Gauss points -- the integral
 * the locally corrected weights reproduce exactly.  The element integrals are
 * done here without the corrected weights:
 *   - x_i off the element: error-controlled adaptive subdivision (two
 *     collapsed Gauss rules of different order must agree, else split);
 *   - x_i on the element: the integral over the element minus the ball
 *     |y - x_i| < eps, in polar coordinates with a logarithmic radial
 *     variable, minus the divergent part h u(x_i)/(2 eps) (h = coefficient of
 *     d2G/dn_x dn_y; the Laplace hypersingular kernel on a smooth surface
 *     diverges exactly like that), extrapolated to eps -> 0 by Richardson:
 *     this is the definition of the Hadamard finite part with a vanishing
 *     spherical neighbourhood (section 2.1).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

void oracle_kernels(const double *x, const double *nx, const double *y, const double *ny, double k,
                    double *out_re_im);

static cplx kcombo(const double *x, const double *nx, const double *y, const double *ny, double k, const cplx c[4])
{
    double v[8];
    oracle_kernels(x, nx, y, ny, k, v);
    cplx G = v[0] + I * v[1], Gy = v[2] + I * v[3], Gx = v[4] + I * v[5], Gxy = v[6] + I * v[7];
    return c[0] * c[2] * G + c[1] * c[2] * Gy + c[0] * c[3] * Gx + c[1] * c[3] * Gxy;
}

/* ---- element geometry: quadratic map on the reference triangle ---- */
static void shape(double s, double t, double N[6], double Ns[6], double Nt[6])
{
    double L0 = 1 - s - t;
    N[0] = L0 * (2 * L0 - 1); N[1] = s * (2 * s - 1); N[2] = t * (2 * t - 1);
    N[3] = 4 * L0 * s; N[4] = 4 * s * t; N[5] = 4 * t * L0;
    Ns[0] = 1 - 4 * L0; Ns[1] = 4 * s - 1; Ns[2] = 0; Ns[3] = 4 * (L0 - s); Ns[4] = 4 * t; Ns[5] = -4 * t;
    Nt[0] = 1 - 4 * L0; Nt[1] = 0; Nt[2] = 4 * t - 1; Nt[3] = -4 * s; Nt[4] = 4 * s; Nt[5] = 4 * (L0 - t);
}

/* position, unit normal (into the body) and area element at (s,t) */
static void geom(const double *el, double s, double t, double y[3], double n[3], double *J)
{
    double N[6], Ns[6], Nt[6], a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    shape(s, t, N, Ns, Nt);
    for (int d = 0; d < 3; ++d) {
        y[d] = 0;
        for (int q = 0; q < 6; ++q) {
            y[d] += N[q] * el[3 * q + d];
            a[d] += Ns[q] * el[3 * q + d];
            b[d] += Nt[q] * el[3 * q + d];
        }
    }
    double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    *J = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    for (int d = 0; d < 3; ++d) n[d] = -c[d] / *J;
}

static double dist3(const double *a, const double *b)
{
    double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

/* distance from x to the element: dense parametric sampling, then a shrinking
 * pattern search around the best sample */
static double elem_dist(const double *el, const double *x)
{
    double best = 1e300, bs = 0, bt = 0, y[3], n[3], J;
    const int G = 24;
    for (int i = 0; i <= G; ++i)
        for (int j = 0; i + j <= G; ++j) {
            double s = (double)i / G, t = (double)j / G;
            geom(el, s, t, y, n, &J);
            double d = dist3(x, y);
            if (d < best) best = d, bs = s, bt = t;
        }
    double h = 1.0 / G;
    while (h > 1e-10) {
        int moved = 0;
        for (int dir = 0; dir < 8; ++dir) {
            double ds = (dir == 0) - (dir == 1) + (dir == 4) - (dir == 5) + (dir == 6) - (dir == 7);
            double dt = (dir == 2) - (dir == 3) + (dir == 4) - (dir == 5) - (dir == 6) + (dir == 7);
            double s = bs + h * ds, t = bt + h * dt;
            if (s < 0 || t < 0 || s + t > 1) continue;
            geom(el, s, t, y, n, &J);
            double d = dist3(x, y);
            if (d < best) {
                best = d, bs = s, bt = t;
                moved = 1;
            }
        }
        if (!moved) h *= 0.5;
    }
    return best;
}

static double longest_side(const double *el)
{
    double L = 0;
    for (int a = 0; a < 3; ++a) {
        double d = dist3(el + 3 * a, el + 3 * ((a + 1) % 3));
        if (d > L) L = d;
    }
    return L;
}

/* ---- 1-D Gauss-Legendre on [0,1] ---- */
static void gl01(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 1;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1, p1 = z;
            for (int l = 2; l <= n; ++l) {
                double p2 = ((2.0 * l - 1) * z * p1 - (l - 1.0) * p0) / l;
                p0 = p1;
                p1 = p2;
            }
            pp = n * (z * p1 - p0) / (z * z - 1);
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = 0.5 * (1 - z);
        w[i] = 1.0 / ((1 - z * z) * pp * pp);
    }
}

/* ---- the interpolant: u~(s,t) = sum_n a_n phi_n with V a = u_D ---- */
static void phis(double s, double t, double p[6])
{
    p[0] = 1; p[1] = s; p[2] = t; p[3] = s * s; p[4] = s * t; p[5] = t * t;
}

static void solve6(double A[6][6], cplx b[6])
{
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        for (int r = c + 1; r < 6; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        for (int q = 0; q < 6; ++q) {
            double tmp = A[c][q];
            A[c][q] = A[piv][q];
            A[piv][q] = tmp;
        }
        cplx tb = b[c];
        b[c] = b[piv];
        b[piv] = tb;
        for (int r = c + 1; r < 6; ++r) {
            double f = A[r][c] / A[c][c];
            for (int q = c; q < 6; ++q) A[r][q] -= f * A[c][q];
            b[r] -= f * b[c];
        }
    }
    for (int c = 5; c >= 0; --c) {
        cplx s = b[c];
        for (int q = c + 1; q < 6; ++q) s -= A[c][q] * b[q];
        b[c] = s / A[c][c];
    }
}

typedef struct {
    const double *el, *x, *nx;
    double k;
    cplx c[4];
    cplx a[6];  /* interpolant coefficients */
    double *gx6, *gw6, *gx10, *gw10;
} Job;

static cplx ut(const Job *J, double s, double t)
{
    double p[6];
    phis(s, t, p);
    cplx v = 0;
    for (int n = 0; n < 6; ++n) v += J->a[n] * p[n];
    return v;
}

/* collapsed Gauss over the sub-triangle v (reference coords) with an n-point 1-D rule */
static cplx tri_rule(const Job *J, const double v[3][2], int n, const double *gx, const double *gw)
{
    double e1[2] = {v[1][0] - v[0][0], v[1][1] - v[0][1]}, e2[2] = {v[2][0] - v[0][0], v[2][1] - v[0][1]};
    double jac = fabs(e1[0] * e2[1] - e1[1] * e2[0]);
    cplx acc = 0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double u = gx[a], vv = gx[b] * (1 - gx[a]), wq = gw[a] * gw[b] * (1 - gx[a]) * jac;
            double s = v[0][0] + u * e1[0] + vv * e2[0], t = v[0][1] + u * e1[1] + vv * e2[1];
            double y[3], ny[3], Jy;
            geom(J->el, s, t, y, ny, &Jy);
            acc += kcombo(J->x, J->nx, y, ny, J->k, J->c) * ut(J, s, t) * (Jy * wq);
        }
    return acc;
}

static cplx adapt(const Job *J, const double v[3][2], cplx coarse, int depth, double atol)
{
    cplx fine = tri_rule(J, v, 10, J->gx10, J->gw10);
    if (cabs(fine - coarse) <= atol || depth >= 16) return fine;
    double m[3][2];
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 2; ++d) m[a][d] = 0.5 * (v[a][d] + v[(a + 1) % 3][d]);
    double sub[4][3][2] = {{{v[0][0], v[0][1]}, {m[0][0], m[0][1]}, {m[2][0], m[2][1]}},
                           {{m[0][0], m[0][1]}, {v[1][0], v[1][1]}, {m[1][0], m[1][1]}},
                           {{m[2][0], m[2][1]}, {m[1][0], m[1][1]}, {v[2][0], v[2][1]}},
                           {{m[0][0], m[0][1]}, {m[1][0], m[1][1]}, {m[2][0], m[2][1]}}};
    cplx s = 0;
    for (int q = 0; q < 4; ++q) s += adapt(J, (const double(*)[2])sub[q], tri_rule(J, (const double(*)[2])sub[q], 6, J->gx6, J->gw6), depth + 1, 0.25 * atol);
    return s;
}

/* integral over the element minus the ball |y - x| < eps, x = y(s0, t0) */
static cplx excluded_integral(const Job *J, double s0, double t0, double eps, int nth, int nrh,
                              const double *tx, const double *tw, const double *rx, const double *rw)
{
    const double V[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    cplx acc = 0;
    for (int ed = 0; ed < 3; ++ed) {
        const double *pa = V[ed], *pb = V[(ed + 1) % 3];
        double tha = atan2(pa[1] - t0, pa[0] - s0), thb = atan2(pb[1] - t0, pb[0] - s0);
        while (thb < tha) thb += 2 * M_PI;
        for (int q = 0; q < nth; ++q) {
            double th = tha + (thb - tha) * tx[q], wt = (thb - tha) * tw[q];
            double e0 = cos(th), e1 = sin(th);
            /* ray hits the edge pa-pb at rho_hat */
            double ex = pb[0] - pa[0], ey = pb[1] - pa[1];
            double det = e0 * (-ey) - e1 * (-ex);
            double rhat = ((pa[0] - s0) * (-ey) - (pa[1] - t0) * (-ex)) / det;
            /* rho_eps: |y(rho) - x| = eps, bisection (distance grows along the ray) */
            double lo = 0, hi = rhat, y[3], ny[3], Jy;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                geom(J->el, s0 + mid * e0, t0 + mid * e1, y, ny, &Jy);
                if (dist3(y, J->x) < eps) lo = mid; else hi = mid;
                if (hi - lo < 1e-15 * rhat) break;
            }
            double reps = 0.5 * (lo + hi);
            double la = log(reps), lb = log(rhat);
            for (int r = 0; r < nrh; ++r) {
                double lr = la + (lb - la) * rx[r], rho = exp(lr), wr = (lb - la) * rw[r] * rho;
                double s = s0 + rho * e0, t = t0 + rho * e1;
                geom(J->el, s, t, y, ny, &Jy);
                acc += kcombo(J->x, J->nx, y, ny, J->k, J->c) * ut(J, s, t) * (Jy * rho * wr * wt);
            }
        }
    }
    return acc;
}

static cplx self_integral(const Job *J, double s0, double t0, double Lside)
{
    enum { NTH = 64, NRH = 48, NEPS = 5 };
    double tx[NTH], tw[NTH], rx[NRH], rw[NRH];
    gl01(NTH, tx, tw);
    gl01(NRH, rx, rw);
    cplx hyp = J->c[1] * J->c[3];
    cplx u0 = ut(J, s0, t0);
    cplx R[NEPS][NEPS];
    double eps0 = 0.02 * Lside;
    for (int q = 0; q < NEPS; ++q) {
        double eps = eps0 / pow(2.0, q);
        R[q][0] = excluded_integral(J, s0, t0, eps, NTH, NRH, tx, tw, rx, rw) - hyp * u0 / (2 * eps);
    }
    /* Richardson: F(eps) = F + c1 eps + c2 eps^2 + ..., ratio 2 */
    for (int o = 1; o < NEPS; ++o)
        for (int q = 0; q + o < NEPS; ++q) {
            double f = pow(2.0, o);
            R[q][o] = (f * R[q + 1][o - 1] - R[q][o - 1]) / (f - 1);
        }
    return R[0][NEPS - 1];
}

/*
 * out[t] = (A u)_{rows[t]} with the kernel (c0 + c1 d/dn_y)(d0 + d1 d/dn_x) G,
 * free term c.  elem: ne x 6 x 3; pts/nrm/w: the 6 ne nodes (node 6e+g is the
 * g-th Gauss point (s_g, t_g) = gpts[g] of element e).  u, coef, out complex
 * interleaved.
 */
void oracle_corrected_rows(int64_t ne, const double *elem, const double *pts, const double *nrm, const double *w,
                           const double *gpts, const double *u, int64_t m, const int64_t *rows, double k,
                           const double *coef, double free_term, double rel_tol, double *out)
{
    cplx c[4];
    for (int q = 0; q < 4; ++q) c[q] = coef[2 * q] + I * coef[2 * q + 1];
    double gx6[6], gw6[6], gx10[10], gw10[10];
    gl01(6, gx6, gw6);
    gl01(10, gx10, gw10);
    /* Vandermonde of the six Gauss points */
    double V0[6][6];
    for (int g = 0; g < 6; ++g) phis(gpts[2 * g], gpts[2 * g + 1], V0[g]);
    double *Ls = malloc(sizeof(double) * ne), *cen = malloc(sizeof(double) * 3 * ne), *rad = malloc(sizeof(double) * ne);
    for (int64_t e = 0; e < ne; ++e) {
        const double *el = elem + 18 * e;
        Ls[e] = longest_side(el);
        double cc[3] = {0, 0, 0};
        for (int a = 0; a < 6; ++a)
            for (int d = 0; d < 3; ++d) cc[d] += el[3 * a + d] / 6;
        double r = 0;
        for (int a = 0; a < 6; ++a) {
            double dd = dist3(el + 3 * a, cc);
            if (dd > r) r = dd;
        }
        memcpy(cen + 3 * e, cc, sizeof(cc));
        rad[e] = 1.5 * r;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = rows[t];
        const double *x = pts + 3 * i, *nx = nrm + 3 * i;
        cplx acc = free_term * (u[2 * i] + I * u[2 * i + 1]);
        for (int64_t e = 0; e < ne; ++e) {
            const double *el = elem + 18 * e;
            int near = (i / 6 == e);
            if (!near && dist3(x, cen + 3 * e) <= 2 * Ls[e] + rad[e]) near = elem_dist(el, x) <= 2 * Ls[e];
            if (!near) {
                for (int g = 0; g < 6; ++g) {
                    int64_t j = 6 * e + g;
                    acc += w[j] * kcombo(x, nx, pts + 3 * j, nrm + 3 * j, k, c) * (u[2 * j] + I * u[2 * j + 1]);
                }
                continue;
            }
            Job J;
            J.el = el; J.x = x; J.nx = nx; J.k = k;
            for (int q = 0; q < 4; ++q) J.c[q] = c[q];
            double A[6][6];
            memcpy(A, V0, sizeof(A));
            for (int g = 0; g < 6; ++g) J.a[g] = u[2 * (6 * e + g)] + I * u[2 * (6 * e + g) + 1];
            solve6(A, J.a);
            J.gx6 = gx6; J.gw6 = gw6; J.gx10 = gx10; J.gw10 = gw10;
            if (i / 6 == e) {
                int g = (int)(i % 6);
                acc += self_integral(&J, gpts[2 * g], gpts[2 * g + 1], Ls[e]);
            } else {
                const double v[3][2] = {{0, 0}, {1, 0}, {0, 1}};
                cplx coarse = tri_rule(&J, v, 6, gx6, gw6);
                /* absolute tolerance from the size of the plain Gauss-point contribution */
                double scale = 0;
                for (int g = 0; g < 6; ++g) {
                    int64_t j = 6 * e + g;
                    scale += cabs(w[j] * kcombo(x, nx, pts + 3 * j, nrm + 3 * j, k, c)) *
                             cabs(u[2 * j] + I * u[2 * j + 1]);
                }
                acc += adapt(&J, v, coarse, 0, rel_tol * (scale + 1e-300));
            }
        }
        out[2 * t] = creal(acc);
        out[2 * t + 1] = cimag(acc);
    }
    free(Ls);
    free(cen);
    free(rad);
}
