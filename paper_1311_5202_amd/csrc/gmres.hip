// Restarted GMRES for A x = b (paper section 2.2, eq. Axb) with the fast
// directional mat-vec.  x0 = 0; right preconditioning; Arnoldi by classical
// Gram-Schmidt with one re-orthogonalisation pass, all vectors and inner
// products in FP64 on the device; the small Hessenberg least-squares problem
// (Givens rotations) on the host in FP64.  Convergence is tested on the true
// relative residual ||b - A x|| / ||b|| at every restart and at the end.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
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

constexpr int RED_BLOCK = 256;
constexpr int RED_GRID = 512;

// partial[q * RED_GRID + b] = sum over block b's chunk of conj(V_q[i]) w[i]
__global__ __launch_bounds__(RED_BLOCK) void k_multidot(const double2 *__restrict__ V, int64_t ldv,
                                                        const double2 *__restrict__ w, int64_t n,
                                                        double2 *__restrict__ partial)
{
    __shared__ double sre[RED_BLOCK], sim[RED_BLOCK];
    const int q = blockIdx.y;
    const double2 *v = V + (int64_t)q * ldv;
    double re = 0.0, im = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_BLOCK) {
        const double2 a = v[i], b = w[i];
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int s = RED_BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sre[threadIdx.x] += sre[threadIdx.x + s];
            sim[threadIdx.x] += sim[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)q * gridDim.x + blockIdx.x] = make_double2(sre[0], sim[0]);
}

__global__ __launch_bounds__(RED_BLOCK) void k_finish_dot(const double2 *__restrict__ partial, int nb,
                                                          double2 *__restrict__ out)
{
    __shared__ double sre[RED_BLOCK], sim[RED_BLOCK];
    const int q = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int b = threadIdx.x; b < nb; b += RED_BLOCK) {
        re += partial[(int64_t)q * nb + b].x;
        im += partial[(int64_t)q * nb + b].y;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int s = RED_BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sre[threadIdx.x] += sre[threadIdx.x + s];
            sim[threadIdx.x] += sim[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = make_double2(sre[0], sim[0]);
}

// w -= sum_q V_q h_q  (h on the device)
__global__ void k_sub_combo(const double2 *__restrict__ V, int64_t ldv, const double2 *__restrict__ h, int nq,
                            double2 *__restrict__ w, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 acc = w[i];
    for (int q = 0; q < nq; ++q) {
        const double2 v = V[(int64_t)q * ldv + i], c = h[q];
        acc.x -= v.x * c.x - v.y * c.y;
        acc.y -= v.x * c.y + v.y * c.x;
    }
    w[i] = acc;
}

// x += sum_q V_q y_q  (y on the device)
__global__ void k_add_combo(const double2 *__restrict__ V, int64_t ldv, const double2 *__restrict__ y, int nq,
                            double2 *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 acc = x[i];
    for (int q = 0; q < nq; ++q) {
        const double2 v = V[(int64_t)q * ldv + i], c = y[q];
        acc.x += v.x * c.x - v.y * c.y;
        acc.y += v.x * c.y + v.y * c.x;
    }
    x[i] = acc;
}

__global__ void k_scale_copy(const double2 *__restrict__ a, double s, double2 *__restrict__ b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = make_double2(a[i].x * s, a[i].y * s);
}

__global__ void k_sub(const double2 *__restrict__ a, const double2 *__restrict__ b, double2 *__restrict__ c, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = make_double2(a[i].x - b[i].x, a[i].y - b[i].y);
}

__global__ void k_axpy1(const double2 *__restrict__ a, double2 *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = make_double2(x[i].x + a[i].x, x[i].y + a[i].y);
}

__global__ void k_zero(double2 *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_double2(0.0, 0.0);
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

namespace {

struct Work {
    Device &D;
    int64_t n;
    hipStream_t st;
    // h (device) = V[:, 0:nq]^H w
    void multidot(const double2 *V, int nq, const double2 *w, double2 *h)
    {
        hipLaunchKernelGGL(k_multidot, dim3(RED_GRID, nq), dim3(RED_BLOCK), 0, st, V, n, w, n, D.gm_red_c);
        hipLaunchKernelGGL(k_finish_dot, dim3(nq), dim3(RED_BLOCK), 0, st, D.gm_red_c, RED_GRID, h);
    }
    double norm(const double2 *w)
    {
        multidot(w, 1, w, D.gm_h);
        double2 v;
        HIP_CHECK(hipMemcpyAsync(&v, D.gm_h, sizeof(double2), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        return std::sqrt(std::max(v.x, 0.0));
    }
};

}  // namespace

int device_gmres(Plan &P, int op, const double2 *b, double tol, int maxit, int restart, int precond, double2 *x,
                 int *iters, double *relres, double *hist, hipStream_t st)
{
    using cplx = std::complex<double>;
    Device &D = *P.dev;
    const int64_t n = P.N;
    if (precond < 0 || precond > 3) return -7;
    if (precond && !D.bj.inv) build_block_jacobi(P, D);
    if (precond == 2 && (!D.bj.O || D.bj.rank == 0)) return -7;
    if (precond == 3) learned_targets(P);
    const int m = std::max(1, std::min(restart, maxit));
    if ((precond || D.use_graph) && !D.gm_z) {
        HIP_CHECK(hipMalloc(&D.gm_z, sizeof(double2) * n));
        HIP_CHECK(hipMalloc(&D.gm_t, sizeof(double2) * n));
    }
    if (D.gm_m < m) {
        // (re)allocate the Krylov basis
        for (void *p : {(void *)D.gm_V, (void *)D.gm_w, (void *)D.gm_r, (void *)D.gm_h, (void *)D.gm_red_c})
            if (p) (void)hipFree(p);
        HIP_CHECK(hipMalloc(&D.gm_V, sizeof(double2) * (size_t)(m + 1) * n));
        HIP_CHECK(hipMalloc(&D.gm_w, sizeof(double2) * n));
        HIP_CHECK(hipMalloc(&D.gm_r, sizeof(double2) * n));
        HIP_CHECK(hipMalloc(&D.gm_h, sizeof(double2) * (m + 2)));
        HIP_CHECK(hipMalloc(&D.gm_red_c, sizeof(double2) * (size_t)RED_GRID * (m + 2)));
        D.gm_m = m;
    }
    Work W{D, n, st};
    const unsigned g = nblk(n, 256);
    hipLaunchKernelGGL(k_zero, dim3(g), dim3(256), 0, st, x, n);
    const double bnorm = W.norm(b);
    if (!std::isfinite(bnorm)) return -5;
    if (bnorm == 0.0) {
        if (iters) *iters = 0;
        if (relres) *relres = 0.0;
        if (hist) hist[0] = 0.0;
        return 0;
    }
    int it = 0;
    double rel = 1.0;
    if (hist) hist[0] = 1.0;
    std::vector<cplx> H((size_t)(m + 1) * m), cs(m), sn(m), gvec(m + 1), hcol(m + 2);
    // r = b (x0 = 0)
    HIP_CHECK(hipMemcpyAsync(D.gm_r, b, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
    double beta = bnorm;
    int status = -4;
    while (it < maxit) {
        hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, st, D.gm_r, 1.0 / beta, D.gm_V, n);
        std::fill(gvec.begin(), gvec.end(), cplx(0));
        gvec[0] = beta;
        int j = 0;
        bool done = false;
        for (; j < m && it < maxit; ++j) {
            double2 *vj = D.gm_V + (int64_t)j * n;
            if (precond) {
                apply_block_jacobi(P, vj, D.gm_z, st, precond);
                graph_matvec(P, op, D.gm_z, D.gm_w, st);
            } else if (D.use_graph) {
                // fixed buffers so one captured graph serves every step
                hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, st, vj, 1.0, D.gm_z, n);
                graph_matvec(P, op, D.gm_z, D.gm_w, st);
            } else
                device_matvec(P, op, vj, D.gm_w, st);
            // CGS with one re-orthogonalisation
            std::vector<cplx> h(j + 2, cplx(0));
            for (int pass = 0; pass < 2; ++pass) {
                W.multidot(D.gm_V, j + 1, D.gm_w, D.gm_h);
                hipLaunchKernelGGL(k_sub_combo, dim3(g), dim3(256), 0, st, D.gm_V, n, D.gm_h, j + 1, D.gm_w, n);
                std::vector<double2> hv(j + 1);
                HIP_CHECK(hipMemcpyAsync(hv.data(), D.gm_h, sizeof(double2) * (j + 1), hipMemcpyDeviceToHost, st));
                HIP_CHECK(hipStreamSynchronize(st));
                for (int q = 0; q <= j; ++q) h[q] += cplx(hv[q].x, hv[q].y);
            }
            const double hn = W.norm(D.gm_w);
            h[j + 1] = hn;
            ++it;
            for (int q = 0; q <= j + 1; ++q)
                if (!std::isfinite(h[q].real()) || !std::isfinite(h[q].imag())) return -5;
            // apply previous rotations
            for (int q = 0; q < j; ++q) {
                const cplx a = h[q], bb = h[q + 1];
                h[q] = std::conj(cs[q]) * a + std::conj(sn[q]) * bb;
                h[q + 1] = -sn[q] * a + cs[q] * bb;
            }
            // new rotation zeroing h[j+1]
            const double den = std::sqrt(std::norm(h[j]) + std::norm(h[j + 1]));
            if (den == 0.0) return -6;
            cs[j] = h[j] / den;
            sn[j] = h[j + 1] / den;
            h[j] = den;
            h[j + 1] = 0.0;
            const cplx g0 = gvec[j];
            gvec[j] = std::conj(cs[j]) * g0;
            gvec[j + 1] = -sn[j] * g0;
            for (int q = 0; q <= j; ++q) H[(size_t)q + (size_t)j * (m + 1)] = h[q];
            rel = std::abs(gvec[j + 1]) / bnorm;
            if (hist) hist[it] = rel;
            if (rel <= tol) {
                done = true;
                ++j;
                break;
            }
            if (hn == 0.0) {
                // exact invariant subspace: the solution is in the current space
                done = true;
                ++j;
                break;
            }
            hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, st, D.gm_w, 1.0 / hn, D.gm_V + (int64_t)(j + 1) * n, n);
        }
        // y = H^{-1} g (upper triangular j x j)
        std::vector<cplx> y(j);
        for (int q = j - 1; q >= 0; --q) {
            cplx s = gvec[q];
            for (int t = q + 1; t < j; ++t) s -= H[(size_t)q + (size_t)t * (m + 1)] * y[t];
            y[q] = s / H[(size_t)q + (size_t)q * (m + 1)];
        }
        std::vector<double2> yd(j);
        for (int q = 0; q < j; ++q) yd[q] = make_double2(y[q].real(), y[q].imag());
        HIP_CHECK(hipMemcpyAsync(D.gm_h, yd.data(), sizeof(double2) * j, hipMemcpyHostToDevice, st));
        if (precond) {
            // x += M (V y)
            hipLaunchKernelGGL(k_zero, dim3(g), dim3(256), 0, st, D.gm_t, n);
            hipLaunchKernelGGL(k_add_combo, dim3(g), dim3(256), 0, st, D.gm_V, n, D.gm_h, j, D.gm_t, n);
            apply_block_jacobi(P, D.gm_t, D.gm_z, st, precond);
            hipLaunchKernelGGL(k_axpy1, dim3(g), dim3(256), 0, st, D.gm_z, x, n);
        } else
            hipLaunchKernelGGL(k_add_combo, dim3(g), dim3(256), 0, st, D.gm_V, n, D.gm_h, j, x, n);
        // true residual
        graph_matvec(P, op, x, D.gm_w, st);
        hipLaunchKernelGGL(k_sub, dim3(g), dim3(256), 0, st, b, D.gm_w, D.gm_r, n);
        beta = W.norm(D.gm_r);
        rel = beta / bnorm;
        if (!std::isfinite(rel)) return -5;
        if (rel <= tol * (1.0 + 1e-6)) {
            status = 0;
            break;
        }
        if (done && rel > tol) {
            // the recurrence estimate met tol but the true residual did not; keep restarting
        }
    }
    HIP_CHECK(hipStreamSynchronize(st));
    if (iters) *iters = it;
    if (relres) *relres = rel;
    return status;
}

}  // namespace fdbem
