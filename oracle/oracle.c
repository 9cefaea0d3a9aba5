/*
 * Oracle for the Burton-Miller Nystrom summations -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct FP64 CPU code.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may call it; the
 * product library never links, loads or imports anything here, and nothing
 * here is shared with the GPU path.
 *
 * What it computes (paper section 2 and the summation of section 5.1):
 *   - the fundamental solution G = exp(ikr)/(4 pi r) of the Helmholtz
 *     equation and its normal derivatives dG/dn_y, dG/dn_x, d2G/dn_x dn_y
 *     (eq. fundsol and the operators of eq. operator), obtained by direct
 *     differentiation of G with d = x - y, r = |d|;
 *   - the point-kernel sum  p_i = sum_{j != i} w_j K(x_i, y_j) u_j  for a
 *     kernel K = (c0 + c1 d/dn_y)(d0 + d1 d/dn_x) G: with (c0,c1,d0,d1) =
 *     (0,1,1,alpha) this is the H matrix row of eq. eq_hmat, (1,0,1,alpha)
 *     the G matrix row of eq. eq_gmat, (1,alpha,1,0) the test kernel of the
 *     particle summation of section 5.1 (eq. eq_sum).  This is the
 *     "straightforward summation" the paper compares its fast algorithm with.
 *
 * Parity pins live in tests/test_oracle_*.py.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>

typedef double complex cplx;

/* All four kernels at one (x, n_x) <- (y, n_y) pair.
 * out[0] = G, out[1] = dG/dn_y, out[2] = dG/dn_x, out[3] = d2G/dn_x dn_y. */
void oracle_kernels(const double *x, const double *nx, const double *y, const double *ny,
                    double k, double *out_re_im)
{
    double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double dnx = d[0] * nx[0] + d[1] * nx[1] + d[2] * nx[2];
    double dny = d[0] * ny[0] + d[1] * ny[1] + d[2] * ny[2];
    double nn = nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2];
    cplx ik = I * k;
    cplx G = cexp(ik * r) / (4.0 * M_PI * r);
    /* grad_y G = G'(r) * (-d/r),  G'(r) = G (ik - 1/r) */
    cplx Gy = -G * (ik - 1.0 / r) * dny / r;
    /* grad_x G = G'(r) * (d/r) */
    cplx Gx = G * (ik - 1.0 / r) * dnx / r;
    /* dG/dn_y = f(r) (d.n_y) with f = G (1/r - ik)/r; differentiate along n_x:
       f'(r) (d.n_x)(d.n_y)/r + f(r) (n_x.n_y) */
    cplx f = G * (1.0 / r - ik) / r;
    cplx fp_over_r = G * (k * k / (r * r) + 3.0 * ik / (r * r * r) - 3.0 / (r * r * r * r));
    cplx Gxy = fp_over_r * dnx * dny + f * nn;
    cplx v[4] = {G, Gy, Gx, Gxy};
    for (int a = 0; a < 4; ++a) {
        out_re_im[2 * a] = creal(v[a]);
        out_re_im[2 * a + 1] = cimag(v[a]);
    }
}

static inline cplx kernel_combo(const double *x, const double *nx, const double *y, const double *ny,
                                double k, cplx c0, cplx c1, cplx d0, cplx d1)
{
    double v[8];
    oracle_kernels(x, nx, y, ny, k, v);
    cplx G = v[0] + I * v[1], Gy = v[2] + I * v[3], Gx = v[4] + I * v[5], Gxy = v[6] + I * v[7];
    return c0 * d0 * G + c1 * d0 * Gy + c0 * d1 * Gx + c1 * d1 * Gxy;
}

/*
 * Dense point-kernel sum over selected target rows.
 *   pts  : (n, 3) node positions, nrm : (n, 3) unit normals, w : (n) weights
 *   u    : (n) complex densities as interleaved (re, im)
 *   rows : (m) target node indices; the j == rows[t] term is excluded
 *   coef : c0, c1, d0, d1 as interleaved (re, im)
 *   out  : (m) complex, interleaved
 */
void oracle_dense_rows(int64_t n, const double *pts, const double *nrm, const double *w,
                       const double *u, int64_t m, const int64_t *rows, double k,
                       const double *coef, double *out)
{
    cplx c0 = coef[0] + I * coef[1], c1 = coef[2] + I * coef[3];
    cplx d0 = coef[4] + I * coef[5], d1 = coef[6] + I * coef[7];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = rows[t];
        cplx acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            cplx K = kernel_combo(pts + 3 * i, nrm + 3 * i, pts + 3 * j, nrm + 3 * j, k, c0, c1, d0, d1);
            acc += w[j] * K * (u[2 * j] + I * u[2 * j + 1]);
        }
        out[2 * t] = creal(acc);
        out[2 * t + 1] = cimag(acc);
    }
}

/* Dense matrix rows: mat[t, j] = w_j K(x_rows[t], y_j), zero on j == rows[t]. */
void oracle_dense_matrix(int64_t n, const double *pts, const double *nrm, const double *w,
                         int64_t m, const int64_t *rows, double k, const double *coef, double *mat)
{
    cplx c0 = coef[0] + I * coef[1], c1 = coef[2] + I * coef[3];
    cplx d0 = coef[4] + I * coef[5], d1 = coef[6] + I * coef[7];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = rows[t];
        for (int64_t j = 0; j < n; ++j) {
            cplx K = 0.0;
            if (j != i)
                K = w[j] * kernel_combo(pts + 3 * i, nrm + 3 * i, pts + 3 * j, nrm + 3 * j, k, c0, c1, d0, d1);
            mat[2 * (t * n + j)] = creal(K);
            mat[2 * (t * n + j) + 1] = cimag(K);
        }
    }
}

int oracle_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}
