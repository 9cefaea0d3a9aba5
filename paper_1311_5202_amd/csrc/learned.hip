// Learned coupling correction of the block-Jacobi preconditioner.
//
// Blocks b (octree leaves cut into pieces of at most 64 points) get an
// overlapping point set E_b: the block's own points first, then up to 64 of
// the nearest points among its leaf's direct-sum sources (ne_b <= 128).  The
// preconditioner applied to v is
//   z_b = A_bb^{-1} v_b + U_b (W_b^H v_{E_b}),
// with U_b (n_b x RANK) and W_b (ne_b x RANK) produced row by row by a small
// network from features of the pair (block b, point j of E_b).  The network
// output is fixed during a solve, so z depends linearly on v and plain
// right-preconditioned GMRES stays valid; with no network loaded only the
// block-Jacobi part is applied.
//
// Training target (generated from the operator itself): the rows of block b of
// the inverse of the corrected operator restricted to E_b,
// R_b = [(A|E_b)^{-1}]_{b, E_b} (restricted additive Schwarz rows), with
//   loss = sum_b w_b || [A_bb^{-1} 0] + U_b W_b^H - R_b ||_F^2,
//   w_b = 1 / ||R_b - [A_bb^{-1} 0]||_F^2  (0 when that is <= 1e-12 ||R_b||_F^2).
// Pair features (NF = 12): k (x_j - c_b) (3), n_j (3), w_j k^2, n_b / 64,
// k r_b (block radius), [j in block b], Re/Im (A_bb^{-1})_jj for j in the block.
// Network: NF -> NH (tanh) -> 4 RANK outputs per pair row: Re/Im of row j of
// U (read for the block's own points) then Re/Im of row j of W.
// Features, forward, loss gradient, backward and Adam run in the kernels below.
#include <hip/hip_runtime.h>

#include <algorithm>
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

namespace lp {

constexpr int NF = 12, NH = 32, RANK = 4, NO = 4 * RANK;
constexpr int NPAR = NF * NH + NH + NH * NO + NO;  // W1 (NH x NF), b1, W2 (NO x NH), b2
constexpr int EXT = 128;      // points of an overlapping set E_b
constexpr int OVERLAP = 64;   // points added to a block
constexpr int BMAX = 64;

__device__ __forceinline__ double2 zmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zdiv(double2 a, double2 b)
{
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

__device__ inline double2 h_kernel(const double *x, const double *nx, const double *y, const double *ny, double k,
                                   double ik)
{
    const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2), ir = 1.0 / r;
    const double dnx = (d0 * nx[0] + d1 * nx[1] + d2 * nx[2]) * ir;
    const double dny = (d0 * ny[0] + d1 * ny[1] + d2 * ny[2]) * ir;
    const double nn = nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2];
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const double g = ir * 0.07957747154594767;
    const double2 G = make_double2(cs * g, sn * g);
    const double2 a = make_double2(ir, -k);
    const double2 q = make_double2(k * k - 3.0 * ir * ir, 3.0 * k * ir);
    const double p = dnx * dny, f = nn * ir;
    const double2 B = make_double2(q.x * p + a.x * f, q.y * p + a.y * f);
    return zmul(G, make_double2(a.x * dny - B.y * ik, a.y * dny + B.x * ik));
}

// assemble the corrected operator on E_b (caller indices ext[b][0..ne), block points first),
// padded with the identity to EXT x EXT, column-major
__global__ void k_ext_assemble(const int *__restrict__ ne_, const int64_t *__restrict__ ext,
                               const double *__restrict__ X, const double *__restrict__ NX, const double *__restrict__ W,
                               const int64_t *__restrict__ crp, const int32_t *__restrict__ cblk,
                               const double2 *__restrict__ cval, double k, double alpha_im, double2 *__restrict__ A)
{
    const int b = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= EXT * EXT) return;
    const int i = e % EXT, j = e / EXT;
    const int ne = ne_[b];
    double2 v = make_double2(i == j ? (i < ne ? 0.5 : 1.0) : 0.0, 0.0);
    if (i < ne && j < ne) {
        const int64_t gi = ext[(size_t)b * EXT + i], gj = ext[(size_t)b * EXT + j];
        if (i != j) {
            const double2 K = h_kernel(X + 3 * gi, NX + 3 * gi, X + 3 * gj, NX + 3 * gj, k, alpha_im);
            v = zadd(v, make_double2(K.x * W[gj], K.y * W[gj]));
        }
        const int32_t ej = (int32_t)(gj / 6);
        for (int64_t q = crp[gi]; q < crp[gi + 1]; ++q)
            if (cblk[q] == ej) {
                v = zadd(v, cval[6 * q + (gj % 6)]);
                break;
            }
    }
    A[(size_t)b * EXT * EXT + e] = v;
}

// in-place Gauss-Jordan inverse of one EXT x EXT matrix per workgroup (global memory)
__global__ __launch_bounds__(256) void k_ext_invert(double2 *__restrict__ Aall, int *__restrict__ fail)
{
    double2 *A = Aall + (size_t)blockIdx.x * EXT * EXT;
    __shared__ int pr[EXT];
    __shared__ int piv;
    __shared__ double2 inv_d;
    const int tid = threadIdx.x;
    for (int c = 0; c < EXT; ++c) {
        if (tid == 0) {
            int p = c;
            double best = -1;
            for (int r = c; r < EXT; ++r) {
                const double2 v = A[r + c * EXT];
                const double m = v.x * v.x + v.y * v.y;
                if (m > best) best = m, p = r;
            }
            piv = p;
            pr[c] = p;
            if (!(best > 0)) atomicExch(fail, 1);
        }
        __syncthreads();
        const int p = piv;
        if (p != c)
            for (int j = tid; j < EXT; j += 256) {
                const double2 t = A[c + j * EXT];
                A[c + j * EXT] = A[p + j * EXT];
                A[p + j * EXT] = t;
            }
        __syncthreads();
        if (tid == 0) inv_d = zdiv(make_double2(1, 0), A[c + c * EXT]);
        __syncthreads();
        const double2 id = inv_d;
        for (int j = tid; j < EXT; j += 256) A[c + j * EXT] = (j == c) ? id : zmul(A[c + j * EXT], id);
        __syncthreads();
        for (int e = tid; e < EXT * EXT; e += 256) {
            const int r = e % EXT, j = e / EXT;
            if (r == c || j == c) continue;
            A[r + j * EXT] = zsub(A[r + j * EXT], zmul(A[r + c * EXT], A[c + j * EXT]));
        }
        __syncthreads();
        for (int r = tid; r < EXT; r += 256)
            if (r != c) A[r + c * EXT] = zmul(make_double2(-A[r + c * EXT].x, -A[r + c * EXT].y), id);
        __syncthreads();
    }
    for (int c = EXT - 1; c >= 0; --c) {
        const int p = pr[c];
        if (p != c)
            for (int r = tid; r < EXT; r += 256) {
                const double2 t = A[r + c * EXT];
                A[r + c * EXT] = A[r + p * EXT];
                A[r + p * EXT] = t;
            }
        __syncthreads();
    }
}

// R_b = rows 0..n_b-1, columns 0..ne_b-1 of the inverted E_b matrix (column-major n_b x ne_b)
__global__ void k_ras_extract(const int *__restrict__ bsize, const int *__restrict__ bne,
                              const int64_t *__restrict__ toff, const double2 *__restrict__ Aall,
                              double2 *__restrict__ T)
{
    const int b = blockIdx.x;
    const int n = bsize[b], ne = bne[b];
    for (int e = threadIdx.x; e < n * ne; e += blockDim.x) {
        const int i = e % n, l = e / n;
        T[toff[b] + e] = Aall[(size_t)b * EXT * EXT + i + (size_t)l * EXT];
    }
}

// pair features: one workgroup per block, thread l for point l of E_b
__global__ __launch_bounds__(EXT) void k_pair_features(const int *__restrict__ bsize, const int *__restrict__ bne,
                                                       const int64_t *__restrict__ ext,
                                                       const int64_t *__restrict__ poff,
                                                       const int64_t *__restrict__ boff, const double *__restrict__ X,
                                                       const double *__restrict__ NX, const double *__restrict__ W,
                                                       const double2 *__restrict__ Binv, double k,
                                                       double *__restrict__ F)
{
    const int b = blockIdx.x, l = threadIdx.x;
    const int n = bsize[b], ne = bne[b];
    const int64_t *e = ext + (size_t)b * EXT;
    __shared__ double c[3], R;
    if (l == 0) {
        c[0] = c[1] = c[2] = 0;
        for (int p = 0; p < n; ++p)
            for (int d = 0; d < 3; ++d) c[d] += X[3 * e[p] + d] / n;
        double r = 0;
        for (int p = 0; p < n; ++p) {
            double s = 0;
            for (int d = 0; d < 3; ++d) s += (X[3 * e[p] + d] - c[d]) * (X[3 * e[p] + d] - c[d]);
            r = fmax(r, sqrt(s));
        }
        R = r;
    }
    __syncthreads();
    if (l >= ne) return;
    const int64_t g = e[l];
    double *f = F + (poff[b] + l) * NF;
    for (int d = 0; d < 3; ++d) f[d] = k * (X[3 * g + d] - c[d]);
    for (int d = 0; d < 3; ++d) f[3 + d] = NX[3 * g + d];
    f[6] = W[g] * k * k;
    f[7] = n / 64.0;
    f[8] = k * R;
    const bool in = l < n;
    f[9] = in ? 1.0 : 0.0;
    const double2 dg = in ? Binv[boff[b] + l + (int64_t)l * n] : make_double2(0, 0);
    f[10] = dg.x;
    f[11] = dg.y;
}

// network forward: O = W2 tanh(W1 f + b1) + b2 per row (H = tanh(...) kept when non-null)
__global__ void k_forward(int64_t np, const double *__restrict__ F, const double *__restrict__ th,
                          double *__restrict__ H, double *__restrict__ O)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const double *W1 = th, *b1 = th + NF * NH, *W2 = b1 + NH, *b2 = W2 + NH * NO;
    const double *f = F + p * NF;
    double h[NH];
#pragma unroll
    for (int a = 0; a < NH; ++a) {
        double s = b1[a];
        for (int q = 0; q < NF; ++q) s += W1[a * NF + q] * f[q];
        h[a] = tanh(s);
        if (H) H[p * NH + a] = h[a];
    }
#pragma unroll
    for (int a = 0; a < NO; ++a) {
        double s = b2[a];
#pragma unroll
        for (int q = 0; q < NH; ++q) s += W2[a * NH + q] * h[q];
        O[p * NO + a] = s;
    }
}

__device__ __forceinline__ double2 out_u(const double *O, int64_t row, int q)
{
    return make_double2(O[row * NO + 2 * q], O[row * NO + 2 * q + 1]);
}
__device__ __forceinline__ double2 out_w(const double *O, int64_t row, int q)
{
    return make_double2(O[row * NO + 2 * RANK + 2 * q], O[row * NO + 2 * RANK + 2 * q + 1]);
}

// per block: D = [Binv 0] + U W^H - R (n x ne); loss_b = w_b ||D||^2; gradients of the outputs
__global__ __launch_bounds__(EXT) void k_block_loss(const int64_t *__restrict__ poff, const int *__restrict__ bsize,
                                                    const int *__restrict__ bne, const int64_t *__restrict__ boff,
                                                    const int64_t *__restrict__ toff,
                                                    const double2 *__restrict__ Binv, const double2 *__restrict__ T,
                                                    const double *__restrict__ O, const double *__restrict__ cw,
                                                    double *__restrict__ dout, double *__restrict__ loss)
{
    __shared__ double2 Ds[BMAX * EXT];
    __shared__ double red[EXT], red2[EXT], red3[EXT];
    const int b = blockIdx.x, t = threadIdx.x;
    const int n = bsize[b], ne = bne[b];
    const int64_t r0 = poff[b];
    double l2 = 0, nrm = 0, tn = 0;
    for (int e = t; e < n * ne; e += EXT) {
        const int i = e % n, l = e / n;
        double2 uw = make_double2(0, 0);
        for (int q = 0; q < RANK; ++q) {
            const double2 u = out_u(O, r0 + i, q), w = out_w(O, r0 + l, q);
            uw = zadd(uw, zmul(u, make_double2(w.x, -w.y)));
        }
        const double2 bi = l < n ? Binv[boff[b] + i + (int64_t)l * n] : make_double2(0, 0);
        const double2 tt = T[toff[b] + e];
        const double2 d = zadd(zsub(bi, tt), uw);
        Ds[e] = d;
        l2 += d.x * d.x + d.y * d.y;
        const double2 r = zsub(tt, bi);
        nrm += r.x * r.x + r.y * r.y;
        tn += tt.x * tt.x + tt.y * tt.y;
    }
    red[t] = l2;
    red2[t] = nrm;
    red3[t] = tn;
    __syncthreads();
    for (int s = EXT / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s], red2[t] += red2[t + s], red3[t] += red3[t + s];
        __syncthreads();
    }
    // w_b, times the block's weight from the method's own GMRES runs when set
    const double scale = (red2[0] > 1e-12 * red3[0] ? 1.0 / red2[0] : 0.0) * (cw ? cw[b] : 1.0);
    if (t == 0) loss[b] = red[0] * scale;
    if (t >= ne) return;
    double *o = dout + (r0 + t) * NO;
    // d/dRe + i d/dIm of |D_il|^2 summed: 2 (D W)_iq for U_iq, 2 (D^H U)_lq for W_lq
    for (int q = 0; q < RANK; ++q) {
        double2 gw = make_double2(0, 0);
        for (int i = 0; i < n; ++i) {
            const double2 d = Ds[i + t * n];
            gw = zadd(gw, zmul(make_double2(d.x, -d.y), out_u(O, r0 + i, q)));
        }
        o[2 * RANK + 2 * q] = 2 * gw.x * scale;
        o[2 * RANK + 2 * q + 1] = 2 * gw.y * scale;
        double2 gu = make_double2(0, 0);
        if (t < n)
            for (int l = 0; l < ne; ++l) gu = zadd(gu, zmul(Ds[t + l * n], out_w(O, r0 + l, q)));
        o[2 * q] = 2 * gu.x * scale;
        o[2 * q + 1] = 2 * gu.y * scale;
    }
}

// backward through the network.  Each workgroup walks chunks of 64 rows,
// stages features, hidden activations and output gradients in LDS and keeps
// per-parameter sums in registers (lane t owns parameters t, t + 64, ...);
// partial sums per workgroup are added in a fixed order by k_grad_sum, so the
// gradient is deterministic.
constexpr int BWP = 64;
constexpr int NACC = (NPAR + BWP - 1) / BWP;
constexpr int BW_GRID = 512;

__global__ __launch_bounds__(BWP) void k_backward(int64_t np, const double *__restrict__ F,
                                                  const double *__restrict__ H, const double *__restrict__ th,
                                                  const double *__restrict__ dout, double *__restrict__ partial)
{
    __shared__ double sf[BWP][NF + 1], sh[BWP][NH + 1], sd[BWP][NO + 1], sdp[BWP][NH + 1];
    const int t = threadIdx.x;
    const double *W2 = th + NF * NH + NH;
    double acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = 0;
    for (int64_t c0 = (int64_t)blockIdx.x * BWP; c0 < np; c0 += (int64_t)gridDim.x * BWP) {
        const int64_t p = c0 + t;
        const bool live = p < np;
        for (int c = 0; c < NF; ++c) sf[t][c] = live ? F[p * NF + c] : 0.0;
        for (int a = 0; a < NO; ++a) sd[t][a] = live ? dout[p * NO + a] : 0.0;
        for (int q = 0; q < NH; ++q) {
            const double h = live ? H[p * NH + q] : 0.0;
            double dh = 0;
            for (int a = 0; a < NO; ++a) dh += W2[a * NH + q] * sd[t][a];
            sh[t][q] = h;
            sdp[t][q] = dh * (1 - h * h);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NACC; ++k) {
            const int i = t + BWP * k;
            double s = 0;
            if (i < NF * NH) {
                const int q = i / NF, c = i % NF;
                for (int pp = 0; pp < BWP; ++pp) s += sdp[pp][q] * sf[pp][c];
            } else if (i < NF * NH + NH) {
                const int q = i - NF * NH;
                for (int pp = 0; pp < BWP; ++pp) s += sdp[pp][q];
            } else if (i < NF * NH + NH + NH * NO) {
                const int j = i - NF * NH - NH, a = j / NH, q = j % NH;
                for (int pp = 0; pp < BWP; ++pp) s += sd[pp][a] * sh[pp][q];
            } else if (i < NPAR) {
                const int a = i - NF * NH - NH - NH * NO;
                for (int pp = 0; pp < BWP; ++pp) s += sd[pp][a];
            }
            acc[k] += s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        const int i = t + BWP * k;
        if (i < NPAR) partial[(size_t)blockIdx.x * NPAR + i] = acc[k];
    }
}

__global__ void k_grad_sum(int nblk, const double *__restrict__ partial, double *__restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAR) return;
    double s = 0;
    for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * NPAR + i];
    grad[i] = s;
}

__global__ void k_adam(double *__restrict__ th, const double *__restrict__ grad, double *__restrict__ m,
                       double *__restrict__ v, double lr, double b1, double b2, double c1, double c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAR) return;
    m[i] = b1 * m[i] + (1 - b1) * grad[i];
    v[i] = b2 * v[i] + (1 - b2) * grad[i] * grad[i];
    th[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + 1e-12);
}

}  // namespace lp

// ---------------------------------------------------------------- host side
struct LearnedNet {
    double *th = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    int step = 0;
};

int learned_num_params() { return lp::NPAR; }

LearnedNet *learned_create(uint64_t seed)
{
    LearnedNet *N = new LearnedNet();
    std::vector<double> th(lp::NPAR, 0.0);
    uint64_t st = seed * 2654435761ull + 12345;
    auto rnd = [&]() {
        st ^= st << 13;
        st ^= st >> 7;
        st ^= st << 17;
        return ((st >> 11) * (1.0 / 9007199254740992.0)) * 2 - 1;
    };
    // Xavier-style initial weights; the output layer starts small so the
    // untrained correction is close to plain block-Jacobi
    for (int i = 0; i < lp::NF * lp::NH; ++i) th[i] = rnd() * std::sqrt(3.0 / lp::NF);
    double *W2 = th.data() + lp::NF * lp::NH + lp::NH;
    for (int i = 0; i < lp::NH * lp::NO; ++i) W2[i] = rnd() * 1e-3;
    for (double **p : {&N->th, &N->grad, &N->m, &N->v}) {
        HIP_CHECK(hipMalloc(p, sizeof(double) * lp::NPAR));
        HIP_CHECK(hipMemset(*p, 0, sizeof(double) * lp::NPAR));
    }
    HIP_CHECK(hipMemcpy(N->th, th.data(), sizeof(double) * lp::NPAR, hipMemcpyHostToDevice));
    return N;
}

void learned_destroy(LearnedNet *N)
{
    if (!N) return;
    for (double *p : {N->th, N->grad, N->m, N->v})
        if (p) (void)hipFree(p);
    delete N;
}

void learned_set_params(LearnedNet *N, const double *th)
{
    HIP_CHECK(hipMemcpy(N->th, th, sizeof(double) * lp::NPAR, hipMemcpyHostToDevice));
}

void learned_get_params(LearnedNet *N, double *th)
{
    HIP_CHECK(hipMemcpy(th, N->th, sizeof(double) * lp::NPAR, hipMemcpyDeviceToHost));
}

// caller-order geometry of a plan on the device (freed by the destructor)
struct GeoUpload {
    double *X = nullptr, *NX = nullptr, *W = nullptr;
    explicit GeoUpload(const Plan &P)
    {
        const int64_t N = P.N;
        std::vector<double> x(3 * N), nx(3 * N), w(N);
        for (int64_t s = 0; s < N; ++s) {
            const int64_t i = P.perm[s];
            x[3 * i] = P.px[s], x[3 * i + 1] = P.py[s], x[3 * i + 2] = P.pz[s];
            nx[3 * i] = P.pnx[s], nx[3 * i + 1] = P.pny[s], nx[3 * i + 2] = P.pnz[s];
            w[i] = P.pw[s];
        }
        HIP_CHECK(hipMalloc(&X, 8 * x.size()));
        HIP_CHECK(hipMalloc(&NX, 8 * nx.size()));
        HIP_CHECK(hipMalloc(&W, 8 * w.size()));
        HIP_CHECK(hipMemcpy(X, x.data(), 8 * x.size(), hipMemcpyHostToDevice));
        HIP_CHECK(hipMemcpy(NX, nx.data(), 8 * nx.size(), hipMemcpyHostToDevice));
        HIP_CHECK(hipMemcpy(W, w.data(), 8 * w.size(), hipMemcpyHostToDevice));
    }
    ~GeoUpload()
    {
        (void)hipFree(X);
        (void)hipFree(NX);
        (void)hipFree(W);
    }
};

static void *plan_alloc(Device &D, size_t bytes, const void *h = nullptr)
{
    void *d = nullptr;
    HIP_CHECK(hipMalloc(&d, std::max<size_t>(bytes, 16)));
    D.allocs.push_back(d);
    D.bytes += bytes;
    if (h && bytes) HIP_CHECK(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice));
    return d;
}

static void block_layout(Device &D, std::vector<int64_t> &bs, std::vector<int> &bn, std::vector<int64_t> &bo)
{
    const int nb = D.bj.n_blocks;
    bs.resize(nb), bn.resize(nb), bo.resize(nb);
    HIP_CHECK(hipMemcpy(bs.data(), D.bj.start, 8 * (size_t)nb, hipMemcpyDeviceToHost));
    HIP_CHECK(hipMemcpy(bn.data(), D.bj.size, 4 * (size_t)nb, hipMemcpyDeviceToHost));
    HIP_CHECK(hipMemcpy(bo.data(), D.bj.off, 8 * (size_t)nb, hipMemcpyDeviceToHost));
}

// overlapping sets E_b: the block, then its nearest points among the direct-sum sources of its leaf
static void ensure_overlap(Plan &P, Device &D)
{
    if (!D.bj.inv) build_block_jacobi(P, D);
    if (D.bj.ext) return;
    std::vector<int64_t> bs, bo;
    std::vector<int> bn;
    block_layout(D, bs, bn, bo);
    const int nb = D.bj.n_blocks;
    std::vector<int> leaf_of(P.N, -1);
    for (size_t t = 0; t < P.leaves.size(); ++t)
        for (int64_t s = P.cubes[P.leaves[t]].start; s < P.cubes[P.leaves[t]].end; ++s) leaf_of[s] = (int)t;
    std::vector<int64_t> ext((size_t)nb * lp::EXT, 0), poff(nb);
    std::vector<int> ne(nb);
    int64_t rows = 0;
    for (int b = 0; b < nb; ++b) {
        const int64_t s0 = bs[b];
        const int n = bn[b];
        double c[3] = {0, 0, 0};
        for (int p = 0; p < n; ++p) c[0] += P.px[s0 + p] / n, c[1] += P.py[s0 + p] / n, c[2] += P.pz[s0 + p] / n;
        std::vector<std::pair<double, int64_t>> cand;
        const int t = leaf_of[s0];
        for (int e = P.p2p_ptr[t]; e < P.p2p_ptr[t + 1]; ++e)
            for (int64_t s = P.p2p_src_start[e]; s < P.p2p_src_end[e]; ++s) {
                if (s >= s0 && s < s0 + n) continue;
                const double d0 = P.px[s] - c[0], d1 = P.py[s] - c[1], d2 = P.pz[s] - c[2];
                cand.push_back({d0 * d0 + d1 * d1 + d2 * d2, s});
            }
        const int extra = std::min({(int)cand.size(), lp::OVERLAP, lp::EXT - n});
        std::partial_sort(cand.begin(), cand.begin() + extra, cand.end());
        for (int p = 0; p < n; ++p) ext[(size_t)b * lp::EXT + p] = P.perm[s0 + p];
        for (int p = 0; p < extra; ++p) ext[(size_t)b * lp::EXT + n + p] = P.perm[cand[p].second];
        ne[b] = n + extra;
        poff[b] = rows;
        rows += ne[b];
    }
    D.bj.ne = (int *)plan_alloc(D, 4 * (size_t)nb, ne.data());
    D.bj.poff = (int64_t *)plan_alloc(D, 8 * (size_t)nb, poff.data());
    D.bj.ext = (int64_t *)plan_alloc(D, 8 * ext.size(), ext.data());
    D.bj.n_pairs = rows;
}

// network inputs of a plan's pair rows and room for the outputs (built once)
static void ensure_features(Plan &P, Device &D)
{
    ensure_overlap(P, D);
    if (D.lt.F) return;
    GeoUpload g(P);
    D.lt.F = (double *)plan_alloc(D, sizeof(double) * D.bj.n_pairs * lp::NF);
    hipLaunchKernelGGL(lp::k_pair_features, dim3(D.bj.n_blocks), dim3(lp::EXT), 0, 0, D.bj.size, D.bj.ne, D.bj.ext,
                       D.bj.poff, D.bj.off, g.X, g.NX, g.W, D.bj.inv, P.k, D.lt.F);
    HIP_CHECK(hipGetLastError());
    D.bj.O = (double *)plan_alloc(D, sizeof(double) * D.bj.n_pairs * lp::NO);
    HIP_CHECK(hipDeviceSynchronize());
}

// training targets R_b, hidden activations and output gradients (built once)
static void ensure_targets(Plan &P, Device &D)
{
    ensure_features(P, D);
    if (D.lt.T) return;
    const int nb = D.bj.n_blocks;
    std::vector<int64_t> bs, bo;
    std::vector<int> bn, ne(nb);
    block_layout(D, bs, bn, bo);
    HIP_CHECK(hipMemcpy(ne.data(), D.bj.ne, 4 * (size_t)nb, hipMemcpyDeviceToHost));
    std::vector<int64_t> toff(nb);
    int64_t tot = 0;
    for (int b = 0; b < nb; ++b) toff[b] = tot, tot += (int64_t)bn[b] * ne[b];
    D.lt.toff = (int64_t *)plan_alloc(D, 8 * (size_t)nb, toff.data());
    D.lt.T = (double2 *)plan_alloc(D, sizeof(double2) * tot);
    GeoUpload g(P);
    // E_b inverses in batches to bound the scratch memory
    const int batch = 1024;
    double2 *dA = nullptr;
    int *dfail = nullptr;
    HIP_CHECK(hipMalloc(&dA, sizeof(double2) * (size_t)batch * lp::EXT * lp::EXT));
    HIP_CHECK(hipMalloc(&dfail, 4));
    HIP_CHECK(hipMemset(dfail, 0, 4));
    for (int b0 = 0; b0 < nb; b0 += batch) {
        const int m = std::min(batch, nb - b0);
        hipLaunchKernelGGL(lp::k_ext_assemble, dim3(lp::EXT * lp::EXT / 256, m), dim3(256), 0, 0, D.bj.ne + b0,
                           D.bj.ext + (size_t)b0 * lp::EXT, g.X, g.NX, g.W, D.corr.rp, D.corr.blk, D.corr.val, P.k,
                           1.0 / P.opt.alpha_k(P.k), dA);
        hipLaunchKernelGGL(lp::k_ext_invert, dim3(m), dim3(256), 0, 0, dA, dfail);
        hipLaunchKernelGGL(lp::k_ras_extract, dim3(m), dim3(256), 0, 0, D.bj.size + b0, D.bj.ne + b0, D.lt.toff + b0,
                           dA, D.lt.T);
        HIP_CHECK(hipGetLastError());
    }
    HIP_CHECK(hipDeviceSynchronize());
    int fail = 0;
    HIP_CHECK(hipMemcpy(&fail, dfail, 4, hipMemcpyDeviceToHost));
    (void)hipFree(dA);
    (void)hipFree(dfail);
    if (fail) throw std::runtime_error("singular overlapping near-field block");
    D.lt.H = (double *)plan_alloc(D, sizeof(double) * D.bj.n_pairs * lp::NH);
    D.lt.dout = (double *)plan_alloc(D, sizeof(double) * D.bj.n_pairs * lp::NO);
    D.lt.loss = (double *)plan_alloc(D, sizeof(double) * nb);
}

// forward, per-block loss, backward and gradient reduction; returns the summed loss
static double loss_grad_core(LearnedNet *Nt, int nb, const int64_t *poff, const int *bsize, const int *bne,
                             const int64_t *boff, const int64_t *toff, int64_t rows, const double *F,
                             const double2 *Binv, const double2 *T, const double *cw, double *H, double *O,
                             double *dout, double *loss)
{
    const int nblk = (int)std::min<int64_t>(lp::BW_GRID, (rows + lp::BWP - 1) / lp::BWP);
    double *partial = nullptr;
    HIP_CHECK(hipMalloc(&partial, sizeof(double) * (size_t)nblk * lp::NPAR));
    HIP_CHECK(hipMemset(dout, 0, sizeof(double) * rows * lp::NO));
    hipLaunchKernelGGL(lp::k_forward, dim3((unsigned)((rows + 127) / 128)), dim3(128), 0, 0, rows, F, Nt->th, H, O);
    hipLaunchKernelGGL(lp::k_block_loss, dim3(nb), dim3(lp::EXT), 0, 0, poff, bsize, bne, boff, toff, Binv, T, O, cw,
                       dout, loss);
    hipLaunchKernelGGL(lp::k_backward, dim3(nblk), dim3(lp::BWP), 0, 0, rows, F, H, Nt->th, dout, partial);
    hipLaunchKernelGGL(lp::k_grad_sum, dim3((lp::NPAR + 255) / 256), dim3(256), 0, 0, nblk, partial, Nt->grad);
    HIP_CHECK(hipGetLastError());
    std::vector<double> l(nb);
    HIP_CHECK(hipMemcpy(l.data(), loss, 8 * (size_t)nb, hipMemcpyDeviceToHost));
    (void)hipFree(partial);
    double s = 0;
    for (double v : l) s += v;
    return s;
}

// loss and gradient on one plan's blocks (gradient left in N->grad)
double learned_loss_grad(LearnedNet *Nt, Plan &P)
{
    Device &D = *P.dev;
    ensure_targets(P, D);
    D.bj.rank = 0;  // the loss overwrites the loaded factors
    return loss_grad_core(Nt, D.bj.n_blocks, D.bj.poff, D.bj.size, D.bj.ne, D.bj.off, D.lt.toff, D.bj.n_pairs, D.lt.F,
                          D.bj.inv, D.lt.T, D.lt.cw, D.lt.H, D.bj.O, D.lt.dout, D.lt.loss);
}

void learned_get_grad(LearnedNet *N, double *g)
{
    HIP_CHECK(hipMemcpy(g, N->grad, sizeof(double) * lp::NPAR, hipMemcpyDeviceToHost));
}

double learned_train_step(LearnedNet *Nt, Plan &P, double lr)
{
    const double loss = learned_loss_grad(Nt, P);
    Nt->step++;
    const double b1 = 0.9, b2 = 0.999;
    hipLaunchKernelGGL(lp::k_adam, dim3((lp::NPAR + 255) / 256), dim3(256), 0, 0, Nt->th, Nt->grad, Nt->m, Nt->v, lr, b1,
                       b2, 1 - std::pow(b1, Nt->step), 1 - std::pow(b2, Nt->step));
    HIP_CHECK(hipGetLastError());
    return loss;
}

// the exact restricted additive Schwarz rows (precond = 3)
void learned_targets(Plan &P) { ensure_targets(P, *P.dev); }

namespace lp {
// energy of the Krylov vectors V_0 .. V_{nv-1} (caller order, length n) on the
// overlapping set of each block: c_b = sum_j sum_{e in E_b} |V_j[e]|^2
__global__ __launch_bounds__(EXT) void k_krylov_energy(int nv, int64_t n, const double2 *__restrict__ V,
                                                       const int *__restrict__ bne, const int64_t *__restrict__ ext,
                                                       double *__restrict__ c)
{
    __shared__ double red[EXT];
    const int b = blockIdx.x, t = threadIdx.x;
    double acc = 0.0;
    if (t < bne[b]) {
        const int64_t i = ext[(int64_t)b * EXT + t];
        for (int j = 0; j < nv; ++j) {
            const double2 v = V[(int64_t)j * n + i];
            acc += v.x * v.x + v.y * v.y;
        }
    }
    red[t] = acc;
    __syncthreads();
    for (int s = EXT / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0) c[b] = red[0];
}
}  // namespace lp

// Block weights of the training loss from the method's own GMRES run: the
// block-Jacobi preconditioned solve of the plan's Burton-Miller operator with
// right-hand side rhs for `iters` steps; c_b is the energy of its Krylov
// vectors (the directions its residuals take) on the block's overlapping set,
// scaled to mean 1.  iters = 0 restores uniform weights.  Returns the number of
// Krylov vectors used.
int learned_weight_blocks(Plan &P, const double2 *rhs, int iters)
{
    Device &D = *P.dev;
    ensure_targets(P, D);
    const int nb = D.bj.n_blocks;
    if (iters <= 0) {
        if (D.lt.cw) HIP_CHECK(hipMemcpy(D.lt.cw, std::vector<double>(nb, 1.0).data(), 8 * (size_t)nb,
                                         hipMemcpyHostToDevice));
        D.lt.cw_active = false;
        return 0;
    }
    double2 *x = nullptr;
    HIP_CHECK(hipMalloc(&x, sizeof(double2) * P.N));
    int it = 0;
    double rel = 0;
    // tolerance 0: the solve runs exactly `iters` steps unless it breaks down
    device_gmres(P, 3, rhs, 1e-300, iters, iters, 1, x, &it, &rel, nullptr, 0);
    HIP_CHECK(hipDeviceSynchronize());
    (void)hipFree(x);
    const int nv = std::max(1, std::min(it, D.gm_m));
    if (!D.lt.cw) D.lt.cw = (double *)plan_alloc(D, 8 * (size_t)nb);
    hipLaunchKernelGGL(lp::k_krylov_energy, dim3(nb), dim3(lp::EXT), 0, 0, nv, P.N, D.gm_V, D.bj.ne, D.bj.ext, D.lt.cw);
    HIP_CHECK(hipGetLastError());
    std::vector<double> c(nb);
    HIP_CHECK(hipMemcpy(c.data(), D.lt.cw, 8 * (size_t)nb, hipMemcpyDeviceToHost));
    double mean = 0;
    for (double v : c) mean += v;
    mean /= std::max(1, nb);
    if (!(mean > 0) || !std::isfinite(mean)) throw std::runtime_error("no Krylov energy on the blocks");
    for (double &v : c) v /= mean;
    HIP_CHECK(hipMemcpy(D.lt.cw, c.data(), 8 * (size_t)nb, hipMemcpyHostToDevice));
    D.lt.cw_active = true;
    return nv;
}

// evaluate the network on a plan and keep its outputs for the preconditioner (precond = 2)
void learned_attach(LearnedNet *Nt, Plan &P)
{
    Device &D = *P.dev;
    ensure_features(P, D);
    hipLaunchKernelGGL(lp::k_forward, dim3((unsigned)((D.bj.n_pairs + 127) / 128)), dim3(128), 0, 0, D.bj.n_pairs,
                       D.lt.F, Nt->th, (double *)nullptr, D.bj.O);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipDeviceSynchronize());
    D.bj.rank = lp::RANK;
}

void learned_detach(Plan &P) { P.dev->bj.rank = 0; }

// raw access for checking the kernels (all device pointers): pair rows
// [poff_b, poff_b + ne_b) of F, block inverses at boff (n_b x n_b) and targets
// at toff (n_b x ne_b), column-major complex
double learned_loss_grad_raw(LearnedNet *Nt, int nb, const int64_t *poff, const int *bsize, const int *bne,
                             const int64_t *boff, const int64_t *toff, int64_t rows, const double *F,
                             const double2 *Binv, const double2 *T, const double *cw)
{
    {
        // the loss kernel holds one block in LDS: check the layout before any launch
        std::vector<int64_t> po(nb), bo(nb), to(nb);
        std::vector<int> bn(nb), be(nb);
        HIP_CHECK(hipMemcpy(po.data(), poff, 8 * (size_t)nb, hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(bn.data(), bsize, 4 * (size_t)nb, hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(be.data(), bne, 4 * (size_t)nb, hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(bo.data(), boff, 8 * (size_t)nb, hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(to.data(), toff, 8 * (size_t)nb, hipMemcpyDeviceToHost));
        for (int b = 0; b < nb; ++b)
            if (bn[b] < 1 || bn[b] > lp::BMAX || be[b] < bn[b] || be[b] > lp::EXT || po[b] < 0 || po[b] + be[b] > rows ||
                bo[b] < 0 || to[b] < 0)
                throw std::invalid_argument("block " + std::to_string(b) +
                                            ": needs 1 <= n <= 64, n <= ne <= 128 and rows inside the feature array");
    }
    double *H = nullptr, *O = nullptr, *dout = nullptr, *loss = nullptr;
    HIP_CHECK(hipMalloc(&H, sizeof(double) * rows * lp::NH));
    HIP_CHECK(hipMalloc(&O, sizeof(double) * rows * lp::NO));
    HIP_CHECK(hipMalloc(&dout, sizeof(double) * rows * lp::NO));
    HIP_CHECK(hipMalloc(&loss, sizeof(double) * nb));
    double s = 0;
    try {
        s = loss_grad_core(Nt, nb, poff, bsize, bne, boff, toff, rows, F, Binv, T, cw, H, O, dout, loss);
    } catch (...) {
        for (void *p : {(void *)H, (void *)O, (void *)dout, (void *)loss}) (void)hipFree(p);
        throw;
    }
    for (void *p : {(void *)H, (void *)O, (void *)dout, (void *)loss}) (void)hipFree(p);
    return s;
}

}  // namespace fdbem
