// Block-Jacobi preconditioner on the corrected near field, and the learned
// low-rank correction applied on top of it.
//
// Blocks are the octree leaves (split into pieces of at most 64 points in
// tree order).  Block b holds A_bb = (1/2) I + [w_j K(x_i, y_j)]_{i != j} +
// (correction table entries inside the block) of the sound-hard operator
// BM_H, inverted in FP64 by Gauss-Jordan with partial pivoting, one
// wavefront per block.  The apply is z_b = A_bb^{-1} v_b (+ U_b (V_b^H v_b)
// with the learned factors when they are loaded), caller node order.
#include <hip/hip_runtime.h>

#include <algorithm>
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

namespace {

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

// dG/dn_y + alpha d2G/dn_x dn_y, alpha = i ik
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

constexpr int BJ_MAX = 64;

// one wavefront per block: assemble A_bb (column-major in LDS), invert in place
__global__ __launch_bounds__(64) void k_bj_build(const int64_t *__restrict__ bstart, const int *__restrict__ bsize,
                                                 const int64_t *__restrict__ boff, const int64_t *__restrict__ perm,
                                                 const double *__restrict__ X, const double *__restrict__ NX,
                                                 const double *__restrict__ W, const int64_t *__restrict__ crp,
                                                 const int32_t *__restrict__ cblk, const double2 *__restrict__ cval,
                                                 double k, double alpha_im, double2 *__restrict__ inv,
                                                 int *__restrict__ fail)
{
    __shared__ double2 A[BJ_MAX * BJ_MAX];
    __shared__ int64_t ci[BJ_MAX];
    __shared__ int piv_row;
    const int b = blockIdx.x, lane = threadIdx.x;
    const int n = bsize[b];
    const int64_t s0 = bstart[b];
    if (lane < n) ci[lane] = perm[s0 + lane];
    __syncthreads();
    for (int e = lane; e < n * n; e += 64) {
        const int i = e % n, j = e / n;
        const int64_t gi = ci[i], gj = ci[j];
        double2 v = make_double2(i == j ? 0.5 : 0.0, 0.0);
        if (i != j) {
            const double2 K = h_kernel(X + 3 * gi, NX + 3 * gi, X + 3 * gj, NX + 3 * gj, k, alpha_im);
            v = zadd(v, make_double2(K.x * W[gj], K.y * W[gj]));
        }
        // correction entry (gi, gj): element gj / 6 in the row's blocks
        const int32_t ej = (int32_t)(gj / 6);
        for (int64_t q = crp[gi]; q < crp[gi + 1]; ++q)
            if (cblk[q] == ej) {
                v = zadd(v, cval[6 * q + (gj % 6)]);
                break;
            }
        A[i + j * BJ_MAX] = v;
    }
    __syncthreads();
    // Gauss-Jordan in place with partial pivoting (row swaps recorded in perm_loc)
    __shared__ int pr[BJ_MAX];
    for (int c = 0; c < n; ++c) {
        if (lane == 0) {
            int p = c;
            double best = -1.0;
            for (int r = c; r < n; ++r) {
                const double2 v = A[r + c * BJ_MAX];
                const double m = v.x * v.x + v.y * v.y;
                if (m > best) best = m, p = r;
            }
            piv_row = p;
            pr[c] = p;
            if (!(best > 0.0)) atomicExch(fail, 1);
        }
        __syncthreads();
        const int p = piv_row;
        if (p != c)
            for (int j = lane; j < n; j += 64) {
                const double2 t = A[c + j * BJ_MAX];
                A[c + j * BJ_MAX] = A[p + j * BJ_MAX];
                A[p + j * BJ_MAX] = t;
            }
        __syncthreads();
        const double2 d = A[c + c * BJ_MAX];
        const double2 one = make_double2(1.0, 0.0);
        const double2 inv_d = zdiv(one, d);
        __syncthreads();
        // scale pivot row, with the pivot position becoming 1/d
        for (int j = lane; j < n; j += 64) A[c + j * BJ_MAX] = (j == c) ? inv_d : zmul(A[c + j * BJ_MAX], inv_d);
        __syncthreads();
        // eliminate column c from the other rows
        for (int e = lane; e < n * n; e += 64) {
            const int r = e % n, j = e / n;
            if (r == c) continue;
            const double2 f = A[r + c * BJ_MAX];
            if (j == c)
                continue;
            A[r + j * BJ_MAX] = zsub(A[r + j * BJ_MAX], zmul(f, A[c + j * BJ_MAX]));
        }
        __syncthreads();
        for (int r = lane; r < n; r += 64)
            if (r != c) A[r + c * BJ_MAX] = zmul(make_double2(-A[r + c * BJ_MAX].x, -A[r + c * BJ_MAX].y), inv_d);
        __syncthreads();
    }
    // undo the row swaps as column swaps of the inverse, in reverse order
    for (int c = n - 1; c >= 0; --c) {
        const int p = pr[c];
        if (p != c)
            for (int r = lane; r < n; r += 64) {
                const double2 t = A[r + c * BJ_MAX];
                A[r + c * BJ_MAX] = A[r + p * BJ_MAX];
                A[r + p * BJ_MAX] = t;
            }
        __syncthreads();
    }
    for (int e = lane; e < n * n; e += 64) {
        const int i = e % n, j = e / n;
        inv[boff[b] + i + (int64_t)j * n] = A[i + j * BJ_MAX];
    }
}

// z = M^-1 v in caller order; one wavefront per block, lane = row.
// mode 1: z_b = A_bb^{-1} v_b; mode 2: plus U_b (W_b^H v_{E_b}) from the
// network outputs O (rank columns; U then W, Re/Im interleaved, NO = 4 rank
// doubles per pair row); mode 3: z_b = R_b v_{E_b} with the stored overlapping
// rows R_b (n_b x ne_b at toff).
constexpr int EXT_MAX = 128, RANK_MAX = 8;

__global__ __launch_bounds__(64) void k_bj_apply(int mode, const int64_t *__restrict__ bstart,
                                                 const int *__restrict__ bsize, const int64_t *__restrict__ boff,
                                                 const int64_t *__restrict__ perm, const double2 *__restrict__ inv,
                                                 const int *__restrict__ bne, const int64_t *__restrict__ ext,
                                                 const int64_t *__restrict__ poff, const double *__restrict__ O,
                                                 int rank, const double2 *__restrict__ R,
                                                 const int64_t *__restrict__ toff, const double2 *__restrict__ v,
                                                 double2 *__restrict__ z)
{
    __shared__ double2 ve[EXT_MAX];
    __shared__ double2 part[RANK_MAX][64];
    __shared__ double2 t[RANK_MAX];
    const int b = blockIdx.x, lane = threadIdx.x;
    const int n = bsize[b];
    const int64_t s0 = bstart[b];
    const int64_t gi = lane < n ? perm[s0 + lane] : 0;
    const int ne = mode >= 2 ? bne[b] : n;
    if (mode >= 2) {
        for (int l = lane; l < ne; l += 64) ve[l] = v[ext[(size_t)b * EXT_MAX + l]];
    } else if (lane < n) {
        ve[lane] = v[gi];
    }
    __syncthreads();
    double2 acc = make_double2(0.0, 0.0);
    if (mode == 3) {
        if (lane < n) {
            const double2 *M = R + toff[b];
            for (int l = 0; l < ne; ++l) acc = zadd(acc, zmul(M[lane + (int64_t)l * n], ve[l]));
        }
    } else {
        if (lane < n) {
            const double2 *M = inv + boff[b];
            for (int j = 0; j < n; ++j) acc = zadd(acc, zmul(M[lane + (int64_t)j * n], ve[j]));
        }
        if (mode == 2 && rank > 0) {
            const int no = 4 * rank;
            const int64_t r0 = poff[b];
            for (int q = 0; q < rank; ++q) {
                double2 s = make_double2(0.0, 0.0);
                for (int l = lane; l < ne; l += 64) {
                    const double *o = O + (r0 + l) * no + 2 * rank + 2 * q;
                    s = zadd(s, zmul(make_double2(o[0], -o[1]), ve[l]));
                }
                part[q][lane] = s;
            }
            __syncthreads();
            if (lane < rank) {
                double2 s = make_double2(0.0, 0.0);
                for (int m = 0; m < 64; ++m) s = zadd(s, part[lane][m]);
                t[lane] = s;
            }
            __syncthreads();
            if (lane < n)
                for (int q = 0; q < rank; ++q) {
                    const double *o = O + (r0 + lane) * no + 2 * q;
                    acc = zadd(acc, zmul(make_double2(o[0], o[1]), t[q]));
                }
        }
    }
    if (lane < n) z[gi] = acc;
}

}  // namespace

void build_block_jacobi(Plan &P, Device &D)
{
    if (!D.corr.val) throw std::invalid_argument("block-Jacobi needs the corrected H table (elements)");
    // blocks: leaves split into pieces of at most BJ_MAX points
    std::vector<int64_t> bs, bo;
    std::vector<int> bn;
    int64_t off = 0;
    for (int id : P.leaves) {
        const Cube &c = P.cubes[id];
        for (int64_t s = c.start; s < c.end; s += BJ_MAX) {
            const int n = (int)std::min<int64_t>(BJ_MAX, c.end - s);
            bs.push_back(s);
            bn.push_back(n);
            bo.push_back(off);
            off += (int64_t)n * n;
        }
    }
    const int nb = (int)bs.size();
    auto up = [&](const void *h, size_t bytes) {
        void *d = nullptr;
        HIP_CHECK(hipMalloc(&d, std::max<size_t>(bytes, 16)));
        D.allocs.push_back(d);
        D.bytes += bytes;
        if (bytes && h) HIP_CHECK(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice));
        return d;
    };
    D.bj.n_blocks = nb;
    D.bj.start = (int64_t *)up(bs.data(), 8 * bs.size());
    D.bj.size = (int *)up(bn.data(), 4 * bn.size());
    D.bj.off = (int64_t *)up(bo.data(), 8 * bo.size());
    D.bj.inv = (double2 *)up(nullptr, sizeof(double2) * (size_t)off);
    // caller-order geometry
    const int64_t N = P.N;
    std::vector<double> X(3 * N), NX(3 * N), W(N);
    for (int64_t s = 0; s < N; ++s) {
        const int64_t i = P.perm[s];
        X[3 * i] = P.px[s], X[3 * i + 1] = P.py[s], X[3 * i + 2] = P.pz[s];
        NX[3 * i] = P.pnx[s], NX[3 * i + 1] = P.pny[s], NX[3 * i + 2] = P.pnz[s];
        W[i] = P.pw[s];
    }
    double *dX = nullptr, *dNX = nullptr, *dW = nullptr;
    int *dfail = nullptr;
    HIP_CHECK(hipMalloc(&dX, 8 * X.size()));
    HIP_CHECK(hipMalloc(&dNX, 8 * NX.size()));
    HIP_CHECK(hipMalloc(&dW, 8 * W.size()));
    HIP_CHECK(hipMalloc(&dfail, sizeof(int)));
    HIP_CHECK(hipMemcpy(dX, X.data(), 8 * X.size(), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(dNX, NX.data(), 8 * NX.size(), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(dW, W.data(), 8 * W.size(), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemset(dfail, 0, sizeof(int)));
    hipLaunchKernelGGL(k_bj_build, dim3(nb), dim3(64), 0, 0, D.bj.start, D.bj.size, D.bj.off, D.perm, dX, dNX, dW,
                       D.corr.rp, D.corr.blk, D.corr.val, P.k, 1.0 / P.opt.alpha_k(P.k), D.bj.inv, dfail);
    HIP_CHECK(hipGetLastError());
    int fail = 0;
    HIP_CHECK(hipMemcpy(&fail, dfail, sizeof(int), hipMemcpyDeviceToHost));
    (void)hipFree(dX);
    (void)hipFree(dNX);
    (void)hipFree(dW);
    (void)hipFree(dfail);
    if (fail) throw std::runtime_error("singular near-field block in the block-Jacobi preconditioner");
}

// mode 1: block inverses; 2: block inverses plus the learned coupling; 3: the
// restricted additive Schwarz rows the coupling is trained towards
void apply_block_jacobi(Plan &P, const double2 *v, double2 *z, hipStream_t st, int mode)
{
    Device &D = *P.dev;
    if (mode == 2 && !(D.bj.O && D.bj.rank > 0 && D.bj.rank <= RANK_MAX)) throw std::logic_error("no learned factors");
    if (mode == 3 && !(D.lt.T && D.bj.ext)) throw std::logic_error("overlapping rows not built");
    if (!D.bj.inv) throw std::logic_error("block-Jacobi blocks not built");
    hipLaunchKernelGGL(k_bj_apply, dim3(D.bj.n_blocks), dim3(64), 0, st, mode, D.bj.start, D.bj.size, D.bj.off, D.perm,
                       D.bj.inv, D.bj.ne, D.bj.ext, D.bj.poff, D.bj.O, mode == 2 ? D.bj.rank : 0, D.lt.T, D.lt.toff, v,
                       z);
    HIP_CHECK(hipGetLastError());
}

}  // namespace fdbem
