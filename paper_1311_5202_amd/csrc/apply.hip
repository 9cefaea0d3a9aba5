// HIP kernels and launch sequence of the fast directional Burton-Miller
// mat-vec (paper sections 3.1.2 and 3.2) for gfx950.
//
// One mat-vec, all stream-ordered:
//   permute + weight  s_j = w_j u_perm(j)                  (sorted order)
//   P2P               near field, direct kernel sums        (section 3.2, modification 3)
//   S2M               check potentials of leaf sources, then W = S~^-1 U~^H
//                     (E_up = dG/dn_y for the H sum: modification 1)
//   M2M               bottom-up, compressed M~ per (level, wedge, octant)
//   M2L               per level, K~ or its low-rank factors U^ (V^ x)
//   L2L               top-down, L~ = M~^T
//   L2T               W^T y gives incoming equivalent densities, then
//                     E_dn = G + alpha dG/dn_x at the targets (modification 2)
//   un-permute, free term, near-field correction SpMV (caller order)
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <type_traits>

#include "device.hpp"

namespace fdbem {

#define HIP_CHECK(expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            throw std::runtime_error(std::string("HIP error ") + hipGetErrorString(e_) + " at " + \
                                     __FILE__ + ":" + std::to_string(__LINE__));                 \
    } while (0)

struct OpC {
    double2 cd00, cd10, cd01, cd11;  // products c_a d_b of K = (c0 + c1 d/dn_y)(d0 + d1 d/dn_x) G
    double2 c0, c1, d0, d1;
};
struct OpCf {
    float2 c0, c1, d0, d1;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// complex type and elementary functions for the working precision R
// sin and cos of kr for 0 <= x <~ 1e5: x = q pi/2 + t with q = rint(2x/pi),
// t from two fused multiply-adds against pi/2 split into its nearest double
// and the remainder (absolute error ~1e-16 for q < 2^20), then Taylor series
// of sin and cos on |t| <= pi/4 through t^15 and t^16 (truncation below
// 5e-17) and the quadrant of q.
__device__ __forceinline__ void sincos_kr(double x, double *s, double *c)
{
    const double q = rint(x * 0.63661977236758134308);   // 2/pi
    double t = fma(-q, 1.5707963267948966, x);             // pi/2 rounded to double
    t = fma(-q, 6.123233995736766e-17, t);                 // pi/2 minus that double
    const double t2 = t * t;
    double ps = -1.0 / 1307674368000.0;                    // -1/15!
    ps = fma(ps, t2, 1.0 / 6227020800.0);                  // 1/13!
    ps = fma(ps, t2, -1.0 / 39916800.0);                   // -1/11!
    ps = fma(ps, t2, 1.0 / 362880.0);                      // 1/9!
    ps = fma(ps, t2, -1.0 / 5040.0);                       // -1/7!
    ps = fma(ps, t2, 1.0 / 120.0);                         // 1/5!
    ps = fma(ps, t2, -1.0 / 6.0);                          // -1/3!
    const double sn = fma(ps * t2, t, t);
    double pc = 1.0 / 20922789888000.0;                    // 1/16!
    pc = fma(pc, t2, -1.0 / 87178291200.0);                // -1/14!
    pc = fma(pc, t2, 1.0 / 479001600.0);                   // 1/12!
    pc = fma(pc, t2, -1.0 / 3628800.0);                    // -1/10!
    pc = fma(pc, t2, 1.0 / 40320.0);                       // 1/8!
    pc = fma(pc, t2, -1.0 / 720.0);                        // -1/6!
    pc = fma(pc, t2, 1.0 / 24.0);                          // 1/4!
    pc = fma(pc, t2, -0.5);                                // -1/2!
    const double cn = fma(pc, t2, 1.0);
    const int n = ((int)q) & 3;                              // q < 2^31 for the kr of any plan
    const double a = (n & 1) ? cn : sn, b = (n & 1) ? sn : cn;
    *s = (n & 2) ? -a : a;
    *c = ((n + 1) & 2) ? -b : b;
}

template <typename R> struct Cx;
template <> struct Cx<double> {
    using T = double2;
    __device__ static T mk(double a, double b) { return make_double2(a, b); }
    __device__ static void sc(double x, double *s, double *c) { sincos_kr(x, s, c); }
    __device__ static double rs(double x) { return rsqrt(x); }
};
template <> struct Cx<float> {
    using T = float2;
    __device__ static T mk(float a, float b) { return make_float2(a, b); }
    __device__ static void sc(float x, float *s, float *c) { sincosf(x, s, c); }
    __device__ static float rs(float x) { return rsqrtf(x); }
};
__device__ __forceinline__ double2 to64(double2 a) { return a; }
__device__ __forceinline__ double2 to64(float2 a) { return make_double2(a.x, a.y); }
template <typename C> __device__ __forceinline__ C from64(double2 a);
template <> __device__ __forceinline__ double2 from64<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 from64<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }

constexpr double kInv4Pi = 0.07957747154594767;  // 1/(4 pi)

// Full kernel K(x <- y) with normals at both ends.
__device__ __forceinline__ double2 kernel_full(double dx, double dy, double dz, double nxx, double nxy, double nxz,
                                               double nyx, double nyy, double nyz, double k, const OpC &c)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double r = sqrt(r2);
    const double ir = 1.0 / r;
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const double g = ir * kInv4Pi;
    const double2 G = make_double2(cs * g, sn * g);
    const double dnx = (dx * nxx + dy * nxy + dz * nxz) * ir;  // (d.n_x)/r
    const double dny = (dx * nyx + dy * nyy + dz * nyz) * ir;  // (d.n_y)/r
    const double nn = nxx * nyx + nxy * nyy + nxz * nyz;
    const double2 a = make_double2(ir, -k);                     // 1/r - ik
    const double2 q = make_double2(k * k - 3.0 * ir * ir, 3.0 * k * ir);
    double2 t = c.cd00;
    t = cadd(t, cmul(c.cd10, cscale(a, dny)));
    t = cadd(t, cmul(c.cd01, cscale(a, -dnx)));
    const double2 hx = cadd(cscale(q, dnx * dny), cscale(a, nn * ir));
    t = cadd(t, cmul(c.cd11, hx));
    return cmul(G, t);
}

// Source-side kernel (c0 + c1 d/dn_y) G at a point x without normal.
template <typename R, typename O>
__device__ __forceinline__ typename Cx<R>::T kernel_src(R dx, R dy, R dz, R nyx, R nyy, R nyz, R k, const O &c)
{
    using C = typename Cx<R>::T;
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ir = Cx<R>::rs(r2);
    const R r = r2 * ir;
    R sn, cs;
    Cx<R>::sc(k * r, &sn, &cs);
    const R g = ir * (R)kInv4Pi;
    const C G = Cx<R>::mk(cs * g, sn * g);
    const R dny = (dx * nyx + dy * nyy + dz * nyz) * ir;
    const C a = Cx<R>::mk(ir, -k);
    return cmul(G, cadd(c.c0, cmul(c.c1, cscale(a, dny))));
}

// Target-side kernel (d0 + d1 d/dn_x) G from a point y without normal.
template <typename R, typename O>
__device__ __forceinline__ typename Cx<R>::T kernel_tgt(R dx, R dy, R dz, R nxx, R nxy, R nxz, R k, const O &c)
{
    using C = typename Cx<R>::T;
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ir = Cx<R>::rs(r2);
    const R r = r2 * ir;
    R sn, cs;
    Cx<R>::sc(k * r, &sn, &cs);
    const R g = ir * (R)kInv4Pi;
    const C G = Cx<R>::mk(cs * g, sn * g);
    const R dnx = (dx * nxx + dy * nxy + dz * nxz) * ir;
    const C a = Cx<R>::mk(ir, -k);
    return cmul(G, cadd(c.d0, cmul(c.d1, cscale(a, -dnx))));
}

// ---------------------------------------------------------------- kernels
template <typename C>
__global__ void k_fill_zero(C *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i].x = 0, p[i].y = 0;
}

// weighted densities to tree order, also into the last 16 bytes of each
// point's 64-byte near-field record (pn: 8 doubles per point), so that the
// near-field kernel reads a source with one 64-byte record
__global__ void k_permute_in(const double2 *__restrict__ in, const int64_t *__restrict__ perm,
                             const double *__restrict__ w, double2 *__restrict__ dens, double *__restrict__ pn,
                             int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double2 d = cscale(in[perm[i]], w[i]);
        dens[i] = d;
        *(double2 *)(pn + 8 * i + 6) = d;
    }
}

__global__ void k_permute_out(const double2 *__restrict__ res, const int64_t *__restrict__ perm,
                              const double2 *__restrict__ in, double free_term, double2 *__restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    double2 v = res[i];
    if (free_term != 0.0) v = cadd(v, cscale(in[j], free_term));
    out[j] = v;
}

// Near field.  One 64-lane workgroup per target leaf; the leaf's near-list
// source ranges are concatenated (their point indices staged in LDS), so no
// slice idles at the end of a short range, and its targets run in blocks of
// up to 64: lane = t + nt q for target t of the nt and source slice q of S =
// 64 / nt, so small leaves still fill the wavefront (cutting a leaf into
// smaller blocks that fill more lanes was slower: more distinct sources per
// load instruction); each lane takes two sources per step, and
// the slices are added in order q = 0, 1, .. with cross-lane shuffles.  The
// kernel shape is a template parameter so every operator evaluates only its
// nonzero terms.
struct PN {
    double x, y, z, nx, ny, nz, dre, dim;  // position, normal, weighted density of the current mat-vec
};

enum { OPK_H = 0, OPK_G = 1, OPK_T1 = 2 };

template <int OPK, typename R>
__device__ __forceinline__ typename Cx<R>::T kernel_op(R dx, R dy, R dz, R nxx, R nxy, R nxz, R nyx, R nyy, R nyz, R k,
                                                       R ik)
{
    using C = typename Cx<R>::T;
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ir = Cx<R>::rs(r2);
    const R r = r2 * ir;
    R sn, cs;
    Cx<R>::sc(k * r, &sn, &cs);
    const R g = ir * (R)kInv4Pi;
    const C G = Cx<R>::mk(cs * g, sn * g);
    const C a = Cx<R>::mk(ir, -k);  // 1/r - ik
    C t;
    if (OPK == OPK_H) {
        // dG/dn_y + alpha d2G/dn_x dn_y, alpha = i/k
        const R dnx = (dx * nxx + dy * nxy + dz * nxz) * ir;
        const R dny = (dx * nyx + dy * nyy + dz * nyz) * ir;
        const R nn = nxx * nyx + nxy * nyy + nxz * nyz;
        const C q = Cx<R>::mk(k * k - (R)3 * ir * ir, (R)3 * k * ir);
        const R p = dnx * dny, f = nn * ir;
        const C B = Cx<R>::mk(q.x * p + a.x * f, q.y * p + a.y * f);
        t = Cx<R>::mk(a.x * dny - B.y * ik, a.y * dny + B.x * ik);
    } else if (OPK == OPK_G) {
        // G + alpha dG/dn_x = G [1 - alpha a (d.n_x)/r]
        const R dnx = (dx * nxx + dy * nxy + dz * nxz) * ir;
        t = Cx<R>::mk((R)1 + a.y * dnx * ik, -a.x * dnx * ik);
    } else {
        // G + alpha dG/dn_y = G [1 + alpha a (d.n_y)/r]
        const R dny = (dx * nyx + dy * nyy + dz * nyz) * ir;
        t = Cx<R>::mk((R)1 - a.y * dny * ik, a.x * dny * ik);
    }
    return cmul(G, t);
}

constexpr int P2P_LIST = 2048;  // source indices of a leaf's near list held in LDS per pass

template <int OPK, typename R>
__global__ __launch_bounds__(64) void k_p2p(int n_leaf, const int64_t *__restrict__ ts, const int64_t *__restrict__ te,
                                             const int *__restrict__ ptr,
                                             const int64_t *__restrict__ ss, const int64_t *__restrict__ se,
                                             const PN *__restrict__ pn, double2 *__restrict__ res, double k,
                                             double alpha_im)
{
    using C = typename Cx<R>::T;
    __shared__ int list[P2P_LIST];
    const int leaf = blockIdx.x;
    if (leaf >= n_leaf) return;
    const int lane = threadIdx.x;
    const R kr = (R)k, ik = (R)alpha_im;
    const int e0 = ptr[leaf], e1 = ptr[leaf + 1];
    // the near list's source ranges, concatenated: virtual source v in [0, tot)
    int tot = 0;
    for (int e = e0; e < e1; ++e) tot += (int)(se[e] - ss[e]);
    const int64_t t1 = te[leaf];
    for (int64_t ib = ts[leaf]; ib < t1; ib += 64) {
        // lane = t + nt q: target t of the block's nt (<= 64), source slice q of S = 64 / nt
        const int nt = (int)min((int64_t)64, t1 - ib);
        const int S = 64 / nt;
        const int q = lane / nt, t = lane - q * nt;
        const bool act = q < S;
        const int64_t i = ib + t;
        const PN X = pn[i];
        // the difference in FP64 keeps the phase accurate; the kernel runs in R.
        // The self pair (r = 0) is excluded by a select, not a branch.
        auto term = [&](const PN &Y, int64_t j) {
            C K = kernel_op<OPK, R>((R)(X.x - Y.x), (R)(X.y - Y.y), (R)(X.z - Y.z), (R)X.nx, (R)X.ny, (R)X.nz,
                                    (R)Y.nx, (R)Y.ny, (R)Y.nz, kr, ik);
            return j == i ? Cx<R>::mk(0, 0) : K;
        };
        C acc = Cx<R>::mk(0, 0);
        for (int v0 = 0; v0 < tot; v0 += P2P_LIST) {
            const int nv = min(P2P_LIST, tot - v0);
            __syncthreads();  // the previous pass has read its indices
            for (int e = e0, cum = 0; e < e1 && cum < v0 + nv; ++e) {
                const int64_t a = ss[e];
                const int len = (int)(se[e] - a);
                const int lo = max(v0 - cum, 0), hi = min(v0 + nv - cum, len);
                for (int l = lo + lane; l < hi; l += 64) list[cum + l - v0] = (int)(a + l);
                cum += len;
            }
            __syncthreads();
            if (act) {
                // slice q takes virtual sources q, q + S, .. of the pass, two per step,
                // both loaded before either kernel is evaluated, added in that order
                int v = q;
                for (; v + S < nv; v += 2 * S) {
                    const int j0 = list[v], j1 = list[v + S];
                    const PN Y0 = pn[j0], Y1 = pn[j1];
                    const C d0 = from64<C>(make_double2(Y0.dre, Y0.dim)), d1 = from64<C>(make_double2(Y1.dre, Y1.dim));
                    const C K0 = term(Y0, j0), K1 = term(Y1, j1);
                    acc = cadd(acc, cmul(K0, d0));
                    acc = cadd(acc, cmul(K1, d1));
                }
                if (v < nv) {
                    const int j0 = list[v];
                    const PN Y0 = pn[j0];
                    acc = cadd(acc, cmul(term(Y0, j0), from64<C>(make_double2(Y0.dre, Y0.dim))));
                }
            }
        }
        // slices added in order q = 0, 1, .., S - 1 into the lanes of slice 0
        C sum = acc;
        for (int j = 1; j < S; ++j) {
            const int src = min(t + j * nt, 63);
            const R vx = __shfl(acc.x, src), vy = __shfl(acc.y, src);
            sum.x += vx;
            sum.y += vy;
        }
        if (q == 0) res[ib + t] = to64(sum);
    }
}

constexpr int LEAF_BLOCK = 256;
constexpr int L2T_G = 8;  // leaves per workgroup in S2M and L2T
// S2M: a workgroup takes up to L2T_G leaves of one template.  Check
// potentials phi_g of every leaf's sources at the level's check points
// (template + leaf centre; thread per (leaf, check point)), then x_g = W phi_g
// added to each leaf's outgoing slot (thread per row of W, W read once per
// group).
template <typename R, typename O>
__global__ __launch_bounds__(LEAF_BLOCK) void k_s2m(const int *__restrict__ gptr, const int64_t *__restrict__ start,
                                                    const int64_t *__restrict__ end, const int64_t *__restrict__ slot,
                                                    const int *__restrict__ tmpl, const double *__restrict__ center,
                                                    const int *__restrict__ t_s, const int *__restrict__ t_ny,
                                                    const int64_t *__restrict__ t_yoff,
                                                    const int64_t *__restrict__ t_woff, const double *__restrict__ tY,
                                                    const typename Cx<R>::T *__restrict__ tW,
                                                    const double *__restrict__ X, const double *__restrict__ Y,
                                                    const double *__restrict__ Z, const double *__restrict__ NX,
                                                    const double *__restrict__ NY, const double *__restrict__ NZ,
                                                    const double2 *__restrict__ dens,
                                                    typename Cx<R>::T *__restrict__ od, double k, O c, int max_ny)
{
    using C = typename Cx<R>::T;
    extern __shared__ unsigned char shraw[];
    C *phi = (C *)shraw;  // [L2T_G][max_ny]
    const int tid = threadIdx.x;
    const int ta = gptr[blockIdx.x], ng = gptr[blockIdx.x + 1] - ta;
    const int lev = tmpl[ta];
    const int s = t_s[lev], ny = t_ny[lev];
    const double *Yt = tY + t_yoff[lev];
    const C *W = tW + t_woff[lev];  // element (r, a) at r + a s
    for (int e = tid; e < L2T_G * ny; e += LEAF_BLOCK) {
        const int g = e / ny, a = e - g * ny;
        C acc = Cx<R>::mk(0, 0);
        if (g < ng) {
            const int task = ta + g;
            const double ax = center[3 * task] + Yt[3 * a], ay = center[3 * task + 1] + Yt[3 * a + 1],
                         az = center[3 * task + 2] + Yt[3 * a + 2];
            const int64_t j1 = end[task];
            for (int64_t j = start[task]; j < j1; ++j) {
                const C K = kernel_src<R>((R)(ax - X[j]), (R)(ay - Y[j]), (R)(az - Z[j]), (R)NX[j], (R)NY[j],
                                          (R)NZ[j], (R)k, c);
                acc = cadd(acc, cmul(K, from64<C>(dens[j])));
            }
        }
        phi[g * max_ny + a] = acc;
    }
    __syncthreads();
    for (int r = tid; r < s; r += LEAF_BLOCK) {
        C acc[L2T_G];
#pragma unroll
        for (int g = 0; g < L2T_G; ++g) acc[g] = Cx<R>::mk(0, 0);
        for (int a = 0; a < ny; ++a) {
            const C w = W[r + (int64_t)a * s];
#pragma unroll
            for (int g = 0; g < L2T_G; ++g) acc[g] = cadd(acc[g], cmul(w, phi[g * max_ny + a]));
        }
#pragma unroll
        for (int g = 0; g < L2T_G; ++g)
            if (g < ng) {
                C *o = od + slot[ta + g] + r;
                *o = cadd(*o, acc[g]);
            }
    }
}

// L2T: a workgroup takes up to L2T_G leaves of one template.  First the
// equivalent densities q_g = W^T y_g of every leaf (W read once per group,
// transposed so consecutive threads read consecutive elements), then per
// leaf the targets' sums over the equivalent points, with thread = (target t,
// point slice j) and the slices added in a fixed order.
template <typename R, typename O>
__global__ __launch_bounds__(LEAF_BLOCK) void k_l2t(const int *__restrict__ gptr, const int64_t *__restrict__ start,
                                                    const int64_t *__restrict__ end, const int64_t *__restrict__ slot,
                                                    const int *__restrict__ tmpl, const double *__restrict__ center,
                                                    const int *__restrict__ t_s, const int *__restrict__ t_ny,
                                                    const int64_t *__restrict__ t_yoff,
                                                    const int64_t *__restrict__ t_woff, const double *__restrict__ tY,
                                                    const typename Cx<R>::T *__restrict__ tWt,
                                                    const double *__restrict__ X, const double *__restrict__ Y,
                                                    const double *__restrict__ Z, const double *__restrict__ NX,
                                                    const double *__restrict__ NY, const double *__restrict__ NZ,
                                                    const typename Cx<R>::T *__restrict__ id,
                                                    double2 *__restrict__ res, double k, O c, int max_ny, int max_s)
{
    using C = typename Cx<R>::T;
    extern __shared__ unsigned char shraw[];
    C *q = (C *)shraw;                        // [L2T_G][max_ny]
    C *xs = q + (size_t)L2T_G * max_ny;       // [L2T_G][max_s]
    C *red = xs + (size_t)L2T_G * max_s;      // [LEAF_BLOCK]
    double *ys = (double *)(red + LEAF_BLOCK);  // [3 max_ny]
    const int tid = threadIdx.x;
    const int ta = gptr[blockIdx.x], ng = gptr[blockIdx.x + 1] - ta;
    const int lev = tmpl[ta];
    const int s = t_s[lev], ny = t_ny[lev];
    const double *Yt = tY + t_yoff[lev];
    const C *Wt = tWt + t_woff[lev];  // element (r, a) at a + r ny
    for (int e = tid; e < L2T_G * s; e += LEAF_BLOCK) {
        const int g = e / s, r = e - g * s;
        xs[g * max_s + r] = g < ng ? id[slot[ta + g] + r] : Cx<R>::mk(0, 0);
    }
    for (int e = tid; e < 3 * ny; e += LEAF_BLOCK) ys[e] = Yt[e];
    __syncthreads();
    for (int a = tid; a < ny; a += LEAF_BLOCK) {
        C acc[L2T_G];
#pragma unroll
        for (int g = 0; g < L2T_G; ++g) acc[g] = Cx<R>::mk(0, 0);
        for (int r = 0; r < s; ++r) {
            const C w = Wt[a + (int64_t)r * ny];
#pragma unroll
            for (int g = 0; g < L2T_G; ++g) acc[g] = cadd(acc[g], cmul(w, xs[g * max_s + r]));
        }
#pragma unroll
        for (int g = 0; g < L2T_G; ++g)
            if (g < ng) q[g * max_ny + a] = acc[g];
    }
    __syncthreads();
    for (int g = 0; g < ng; ++g) {
        const int task = ta + g;
        const double cx = center[3 * task], cy = center[3 * task + 1], cz = center[3 * task + 2];
        const C *qg = q + g * max_ny;
        const int64_t i0 = start[task], i1 = end[task];
        for (int64_t ib = i0; ib < i1; ib += LEAF_BLOCK) {
            const int nt = (int)min((int64_t)LEAF_BLOCK, i1 - ib);
            const int S = LEAF_BLOCK / nt;
            const int j = tid / nt, t = tid - j * nt;
            C acc = Cx<R>::mk(0, 0);
            if (j < S) {
                const int64_t i = ib + t;
                const double xi = X[i] - cx, yi = Y[i] - cy, zi = Z[i] - cz;
                const R nxi = (R)NX[i], nyi = (R)NY[i], nzi = (R)NZ[i];
                for (int a = j; a < ny; a += S) {
                    const C K = kernel_tgt<R>((R)(xi - ys[3 * a]), (R)(yi - ys[3 * a + 1]), (R)(zi - ys[3 * a + 2]),
                                              nxi, nyi, nzi, (R)k, c);
                    acc = cadd(acc, cmul(K, qg[a]));
                }
            }
            red[tid] = acc;
            __syncthreads();
            if (tid < nt) {
                C sum = red[tid];
                for (int jj = 1; jj < S; ++jj) sum = cadd(sum, red[tid + jj * nt]);
                res[ib + tid] = cadd(res[ib + tid], to64(sum));
            }
            __syncthreads();
        }
    }
}

// LDS of k_l2t: q and the local densities of L2T_G leaves, the slice sums,
// the check points
template <typename R>
static size_t s2m_shm(const Plan &P)
{
    return sizeof(typename Cx<R>::T) * L2T_G * (size_t)std::max(P.max_Y_leaf, 1);
}
template <typename R>
static size_t l2t_shm(const Plan &P)
{
    const size_t ny = std::max(P.max_Y_leaf, 1), s = std::max(P.max_s, 1);
    return sizeof(typename Cx<R>::T) * (L2T_G * ny + L2T_G * s + LEAF_BLOCK) + sizeof(double) * 3 * ny;
}

// Batched segmented GEMV: out[o] += sum_e op(M_e) in[e]; one block per output slot.
constexpr int GEMV_BLOCK = 128;
constexpr int GEMV_MAXROWS = 2 * GEMV_BLOCK;
enum { TAG_M2M = 0, TAG_M2L = 1, TAG_L2L = 2 };
template <int TAG>
__global__ __launch_bounds__(GEMV_BLOCK) void k_gemv(const int64_t *__restrict__ out_off, const int *__restrict__ ptr,
                                                     const int64_t *__restrict__ in_off,
                                                     const int64_t *__restrict__ mat_off, const int *__restrict__ rank,
                                                     int rows, int cols, int trans, const double2 *__restrict__ mat,
                                                     const double2 *__restrict__ in, double2 *__restrict__ out)
{
    extern __shared__ double2 sh[];
    double2 *xs = sh;          // cols
    double2 *ts = sh + cols;   // low-rank intermediate
    const int o = blockIdx.x, tid = threadIdx.x;
    double2 acc0 = make_double2(0.0, 0.0), acc1 = make_double2(0.0, 0.0);
    const int i0 = tid, i1 = tid + GEMV_BLOCK;
    for (int e = ptr[o]; e < ptr[o + 1]; ++e) {
        __syncthreads();
        const double2 *x = in + in_off[e];
        for (int j = tid; j < cols; j += GEMV_BLOCK) xs[j] = x[j];
        __syncthreads();
        const double2 *M = mat + mat_off[e];
        const int r = rank[e];
        if (r < 0) {
            if (!trans) {
                if (i0 < rows)
                    for (int j = 0; j < cols; ++j) acc0 = cadd(acc0, cmul(M[i0 + (int64_t)j * rows], xs[j]));
                if (i1 < rows)
                    for (int j = 0; j < cols; ++j) acc1 = cadd(acc1, cmul(M[i1 + (int64_t)j * rows], xs[j]));
            } else {
                // M is cols x rows (column-major); use its transpose
                if (i0 < rows)
                    for (int j = 0; j < cols; ++j) acc0 = cadd(acc0, cmul(M[j + (int64_t)i0 * cols], xs[j]));
                if (i1 < rows)
                    for (int j = 0; j < cols; ++j) acc1 = cadd(acc1, cmul(M[j + (int64_t)i1 * cols], xs[j]));
            }
        } else {
            const double2 *U = M;
            const double2 *V = M + (int64_t)rows * r;
            for (int qq = tid; qq < r; qq += GEMV_BLOCK) {
                double2 t = make_double2(0.0, 0.0);
                for (int j = 0; j < cols; ++j) t = cadd(t, cmul(V[qq + (int64_t)j * r], xs[j]));
                ts[qq] = t;
            }
            __syncthreads();
            if (i0 < rows)
                for (int qq = 0; qq < r; ++qq) acc0 = cadd(acc0, cmul(U[i0 + (int64_t)qq * rows], ts[qq]));
            if (i1 < rows)
                for (int qq = 0; qq < r; ++qq) acc1 = cadd(acc1, cmul(U[i1 + (int64_t)qq * rows], ts[qq]));
        }
    }
    const int64_t ob = out_off[o];
    if (i0 < rows) out[ob + i0] = cadd(out[ob + i0], acc0);
    if (i1 < rows) out[ob + i1] = cadd(out[ob + i1], acc1);
}


// M2L over target tiles (see M2LTiles): per chunk the operator is read once
// per row and applied to up to four pairs held in registers; targets
// accumulate in LDS and are written once at the end (no atomics).
// LDS: Y[tile][s] | X[chunk][s] | T[chunk][rmax].
constexpr int M2L_BLOCK = 256;
__global__ __launch_bounds__(M2L_BLOCK) void k_m2l_tile(int s, int rmax, int tile, int chunk, int nseg,
                                                        double2 *__restrict__ part,
                                                        const int64_t *__restrict__ tgt_off,
                                                        const int *__restrict__ tile_ntgt,
                                                        const int *__restrict__ tile_cptr,
                                                        const int64_t *__restrict__ ch_mat,
                                                        const int *__restrict__ ch_rank,
                                                        const int *__restrict__ ch_pptr, const int *__restrict__ pr_tl,
                                                        const int64_t *__restrict__ pr_src,
                                                        const double2 *__restrict__ mat,
                                                        const double2 *__restrict__ od, double2 *__restrict__ id)
{
    extern __shared__ double2 sh[];
    double2 *Y = sh;
    double2 *X = Y + (size_t)tile * s;
    double2 *Tb = X + (size_t)chunk * s;
    const int q = blockIdx.x / nseg, z = blockIdx.x - q * nseg, tid = threadIdx.x;
    const int nt = tile_ntgt[q];
    for (int i = tid; i < nt * s; i += M2L_BLOCK) Y[i] = make_double2(0.0, 0.0);
    // this workgroup's share of the tile's chunks
    const int cb = tile_cptr[q], ce = tile_cptr[q + 1];
    const int c0 = cb + (int)((int64_t)(ce - cb) * z / nseg), c1 = cb + (int)((int64_t)(ce - cb) * (z + 1) / nseg);
    for (int c = c0; c < c1; ++c) {
        const int p0 = ch_pptr[c], n = ch_pptr[c + 1] - p0;
        __syncthreads();
        for (int i = tid; i < n * s; i += M2L_BLOCK) {
            const int p = i / s, j = i - p * s;
            X[i] = od[pr_src[p0 + p] + j];
        }
        __syncthreads();
        const double2 *M = mat + ch_mat[c];
        const int r = ch_rank[c];
        const int G = (n + 3) >> 2;
        if (r < 0) {
            for (int i = tid; i < G * s; i += M2L_BLOCK) {
                const int g = i / s, row = i - g * s;
                double2 a0 = make_double2(0, 0), a1 = a0, a2 = a0, a3 = a0;
                const double2 *x0 = X + (size_t)(4 * g) * s;
                const int np = min(4, n - 4 * g);
                for (int j = 0; j < s; ++j) {
                    const double2 m = M[row + (size_t)j * s];
                    a0 = cadd(a0, cmul(m, x0[j]));
                    if (np > 1) a1 = cadd(a1, cmul(m, x0[s + j]));
                    if (np > 2) a2 = cadd(a2, cmul(m, x0[2 * s + j]));
                    if (np > 3) a3 = cadd(a3, cmul(m, x0[3 * s + j]));
                }
                const int *tl = pr_tl + p0 + 4 * g;
                Y[tl[0] * s + row] = cadd(Y[tl[0] * s + row], a0);
                if (np > 1) Y[tl[1] * s + row] = cadd(Y[tl[1] * s + row], a1);
                if (np > 2) Y[tl[2] * s + row] = cadd(Y[tl[2] * s + row], a2);
                if (np > 3) Y[tl[3] * s + row] = cadd(Y[tl[3] * s + row], a3);
            }
        } else {
            const double2 *U = M, *V = M + (size_t)s * r;
            for (int i = tid; i < G * r; i += M2L_BLOCK) {
                const int g = i / r, qq = i - g * r;
                double2 a0 = make_double2(0, 0), a1 = a0, a2 = a0, a3 = a0;
                const double2 *x0 = X + (size_t)(4 * g) * s;
                const int np = min(4, n - 4 * g);
                for (int j = 0; j < s; ++j) {
                    const double2 m = V[qq + (size_t)j * r];
                    a0 = cadd(a0, cmul(m, x0[j]));
                    if (np > 1) a1 = cadd(a1, cmul(m, x0[s + j]));
                    if (np > 2) a2 = cadd(a2, cmul(m, x0[2 * s + j]));
                    if (np > 3) a3 = cadd(a3, cmul(m, x0[3 * s + j]));
                }
                double2 *t0 = Tb + (size_t)(4 * g) * rmax + qq;
                t0[0] = a0;
                if (np > 1) t0[rmax] = a1;
                if (np > 2) t0[2 * rmax] = a2;
                if (np > 3) t0[3 * rmax] = a3;
            }
            __syncthreads();
            for (int i = tid; i < G * s; i += M2L_BLOCK) {
                const int g = i / s, row = i - g * s;
                double2 a0 = make_double2(0, 0), a1 = a0, a2 = a0, a3 = a0;
                const double2 *t0 = Tb + (size_t)(4 * g) * rmax;
                const int np = min(4, n - 4 * g);
                for (int qq = 0; qq < r; ++qq) {
                    const double2 m = U[row + (size_t)qq * s];
                    a0 = cadd(a0, cmul(m, t0[qq]));
                    if (np > 1) a1 = cadd(a1, cmul(m, t0[rmax + qq]));
                    if (np > 2) a2 = cadd(a2, cmul(m, t0[2 * rmax + qq]));
                    if (np > 3) a3 = cadd(a3, cmul(m, t0[3 * rmax + qq]));
                }
                const int *tl = pr_tl + p0 + 4 * g;
                Y[tl[0] * s + row] = cadd(Y[tl[0] * s + row], a0);
                if (np > 1) Y[tl[1] * s + row] = cadd(Y[tl[1] * s + row], a1);
                if (np > 2) Y[tl[2] * s + row] = cadd(Y[tl[2] * s + row], a2);
                if (np > 3) Y[tl[3] * s + row] = cadd(Y[tl[3] * s + row], a3);
            }
        }
    }
    __syncthreads();
    if (nseg == 1) {
        for (int i = tid; i < nt * s; i += M2L_BLOCK) {
            const int t = i / s, row = i - t * s;
            double2 *o = id + tgt_off[(size_t)q * tile + t] + row;
            *o = cadd(*o, Y[i]);
        }
    } else {
        // partial sums, reduced in a fixed order by k_m2l_reduce
        double2 *pq = part + ((size_t)q * nseg + z) * (size_t)tile * s;
        for (int i = tid; i < nt * s; i += M2L_BLOCK) pq[i] = Y[i];
    }
}

__global__ void k_m2l_reduce(int s, int tile, int nseg, const double2 *__restrict__ part,
                             const int64_t *__restrict__ tgt_off, const int *__restrict__ tile_ntgt,
                             double2 *__restrict__ id)
{
    const int q = blockIdx.x;
    const int nt = tile_ntgt[q];
    for (int i = threadIdx.x; i < nt * s; i += blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int z = 0; z < nseg; ++z) acc = cadd(acc, part[((size_t)q * nseg + z) * (size_t)tile * s + i]);
        const int t = i / s, row = i - t * s;
        double2 *o = id + tgt_off[(size_t)q * tile + t] + row;
        *o = cadd(*o, acc);
    }
}


// M2L by operator chunks: one wavefront per chunk of <= M2LC_CH pairs sharing
// one operator.  Lane = output row; each lane keeps the chunk's pairs in
// registers so every operator element read from cache feeds M2LC_CH complex
// FMAs; sources are staged per wavefront in LDS; results go to the targets
// with FP64 atomic adds (hardware global_atomic_add_f64).
constexpr int M2LC_CH = 16;
constexpr int M2LC_WAVES = 4;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int TAG, bool TRANS, typename R, bool PART>
__global__ __launch_bounds__(64 * M2LC_WAVES) void k_chunks(int n_chunks, int s, int cols, int rmax,
                                                            const int64_t *__restrict__ ch_mat,
                                                            const int *__restrict__ ch_rank,
                                                            const int *__restrict__ ch_pptr,
                                                            const int64_t *__restrict__ pr_tgt,
                                                            const int64_t *__restrict__ pr_src,
                                                            const typename Cx<R>::T *__restrict__ mat,
                                                            const typename Cx<R>::T *__restrict__ od,
                                                            typename Cx<R>::T *id,
                                                            const int64_t *__restrict__ pr_pos,
                                                            typename Cx<R>::T *__restrict__ part)
{
    using C = typename Cx<R>::T;
    extern __shared__ unsigned char shraw[];
    C *sh = (C *)shraw;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * M2LC_WAVES + wv;
    if (c >= n_chunks) return;
    // s: output rows, cols: input length (both equal for M2L)
    C *X = sh + (size_t)wv * (M2LC_CH * cols + M2LC_CH * rmax);
    C *T = X + M2LC_CH * cols;
    const int p0 = ch_pptr[c], n = ch_pptr[c + 1] - p0;
    for (int i = lane; i < n * cols; i += 64) {
        const int p = i / cols, j = i - p * cols;
        X[p * cols + j] = od[pr_src[p0 + p] + j];
    }
    wave_sync();
    const C *M = mat + ch_mat[c];
    const int r = ch_rank[c];
    C acc[M2LC_CH];
    if (r >= 0) {
        // t = V x for every (rank index, pair) item of the chunk
        const C *V = M + (size_t)s * r;
        for (int it = lane; it < r * n; it += 64) {
            const int p = it / r, qq = it - p * r;
            const C *xp = X + p * cols;
            C a = Cx<R>::mk(0, 0);
            for (int j = 0; j < cols; ++j) a = cadd(a, cmul(V[qq + (size_t)j * r], xp[j]));
            T[p * rmax + qq] = a;
        }
        wave_sync();
    }
    for (int row = lane; row < s; row += 64) {
#pragma unroll
        for (int p = 0; p < M2LC_CH; ++p) acc[p] = Cx<R>::mk(0, 0);
        if (r < 0) {
            for (int j = 0; j < cols; ++j) {
                // dense operator s x cols, or its transpose stored cols x s
                const C m = TRANS ? M[j + (size_t)row * cols] : M[row + (size_t)j * s];
#pragma unroll
                for (int p = 0; p < M2LC_CH; ++p)
                    if (p < n) acc[p] = cadd(acc[p], cmul(m, X[p * cols + j]));
            }
        } else {
            for (int qq = 0; qq < r; ++qq) {
                const C m = M[row + (size_t)qq * s];
#pragma unroll
                for (int p = 0; p < M2LC_CH; ++p)
                    if (p < n) acc[p] = cadd(acc[p], cmul(m, T[p * rmax + qq]));
            }
        }
#pragma unroll
        for (int p = 0; p < M2LC_CH; ++p)
            if (p < n) {
                if (PART) {
                    part[pr_pos[p0 + p] * s + row] = acc[p];
                } else {
                    R *o = (R *)(id + pr_tgt[p0 + p] + row);
                    atomicAdd(o, acc[p].x);
                    atomicAdd(o + 1, acc[p].y);
                }
            }
    }
}

// Near-field correction, caller order: out_i += sum over the node's element
// blocks of sum_g val_bg in_{6 e_b + g}.
// Translation chunks on the matrix cores.  One workgroup (4 wavefronts) per
// chunk of <= 16 pairs sharing one operator.  The complex product Y = M X
// (s x cols by cols x 16) is a real product of twice the size with rows
// (Re y_0, Im y_0, Re y_1, ...) and inner index (Re x_0, Im x_0, ...):
// A[2i+c][2j+d] = Re M_ij if c == d, -Im M_ij if (c, d) = (0, 1), Im M_ij if
// (c, d) = (1, 0).  It is evaluated by 16 x 16 x 4 MFMA tiles (16 real rows x
// 4 inner x 16 pairs): lane l holds A[l%16][l/16] and B[l/16][l%16]; result
// register q holds D[4q + l/16][l%16] for the FP64 instruction and
// D[4(l/16) + q][l%16] for the FP32 one.  The sources are staged in LDS in
// the B layout (inner index major, pair fastest); wavefronts split the row
// tiles.  Low-rank operators run V then U with T = V X kept in LDS.  Results
// go to the per-pair scratch (partial-sum schedule).
constexpr int MF_PAIRS = 16;
constexpr int kXcds = 8;  // accelerator complex dies of the MI355X
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <typename R>
struct Mf;
template <>
struct Mf<double> {
    typedef mf_d4 V;
    static __device__ __forceinline__ V mma(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int q, int k4) { return 4 * q + k4; }
    // tile row computed by A row m so that result register q of lane group k4 is row 4 k4 + q
    static __device__ __forceinline__ int rho(int m) { return 4 * (m & 3) + (m >> 2); }
};
template <>
struct Mf<float> {
    typedef mf_f4 V;
    static __device__ __forceinline__ V mma(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int q, int k4) { return 4 * k4 + q; }
    static __device__ __forceinline__ int rho(int m) { return m; }
};

// one real-GEMM sweep over the row tiles: complex A has rows [0, nrow) and
// inner index [0, ncol); element (row, j) at A + row * rs + j * cs (complex
// elements); B holds NT tiles of 16 pairs (row stride 16 NT + 1), and every A
// element loaded feeds NT matrix-core products.  The inner index is split
// into the same four interleaved partial sums for every NT, so a pair's
// result does not depend on NT bit for bit.
// One 16-row tile rt over the real inner range [kb, ke) (kb a multiple of 4).
template <typename R, int NT, typename Store>
__device__ __forceinline__ void mfma_tile(const typename Cx<R>::T *__restrict__ A, int nrow, int64_t rs, int64_t cs,
                                          const R *__restrict__ B, int rt, int kb, int ke, int lane, Store store)
{
    typedef typename Mf<R>::V V;
    constexpr int PW = 16 * NT + 1, U = 4;  // B row stride, padded against LDS bank conflicts
    const int i16 = lane & 15, k4 = lane >> 4;
    const int kmax = ke;
    {
        const int I = rt * 16 + i16, row = I >> 1, ci = I & 1;
        const bool rok = row < nrow;
        const R *arow = (const R *)(A + (rok ? row : 0) * rs);
        V acc[U][NT];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[u][t] = V{0, 0, 0, 0};
        // the inner index of a lane advances by 4 per step: d = k4 & 1 is fixed
        const int d = k4 & 1;
        const R sgn = (ci == 0 && d == 1) ? (R)-1 : (R)1;
        const int sel = ci ^ d;
        int k0 = kb;
        for (; k0 + 4 * U <= kmax; k0 += 4 * U) {
            const int j0 = (k0 + k4) >> 1;
            R x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // always load (arow is row 0 for rows past the end), then mask: no branches
                const R xv = arow[2 * (j0 + 2 * u) * cs + sel];
                x[u] = rok ? xv : (R)0;
            }
            const R *bp = B + (k0 + k4) * PW + i16;
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[u][t] = Mf<R>::mma(sgn * x[u], bp[4 * u * PW + 16 * t], acc[u][t]);
        }
        if (k0 < kmax) {
            // the remaining < 4U inner indices in one masked step (all loads issued together)
            const int j0 = (k0 + k4) >> 1;
            R x[U], bv[U][NT];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int K = k0 + k4 + 4 * u;
                const bool kok = K < kmax;
                const R xv = arow[2 * (kok ? j0 + 2 * u : 0) * cs + sel];
                x[u] = (rok && kok) ? xv : (R)0;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const R b = B[(kok ? K : 0) * PW + 16 * t + i16];
                    bv[u][t] = kok ? b : (R)0;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[u][t] = Mf<R>::mma(sgn * x[u], bv[u][t], acc[u][t]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                R v = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) v += acc[u][t][q];
                const int Io = rt * 16 + Mf<R>::out_row(q, k4);
                store(Io >> 1, Io & 1, t, 16 * t + i16, v);
            }
    }
}

// All row tiles over the full inner range, dealt to the wavefronts.
template <typename R, int NT, typename Store>
__device__ __forceinline__ void mfma_rows(const typename Cx<R>::T *__restrict__ A, int nrow, int ncol, int64_t rs,
                                          int64_t cs, const R *__restrict__ B, int wv, int lane, Store store)
{
    const int n_rt = (2 * nrow + 15) >> 4;
    for (int rt = wv; rt < n_rt; rt += M2LC_WAVES) mfma_tile<R, NT>(A, nrow, rs, cs, B, rt, 0, 2 * ncol, lane, store);
}

// Split of the first low-rank product T = V X over the wavefronts: with
// n_rt < 4 row tiles of T, the inner range 2 cols is cut into ns slices of
// kstep (a multiple of 16) so every wavefront has a (tile, slice) unit; the
// slices are added afterwards in a fixed order.
struct KSplit {
    int n_rt, ns, kstep;
    __device__ KSplit(int r, int cols)
    {
        n_rt = (2 * r + 15) >> 4;
        const int want = (n_rt > 0 && n_rt < M2LC_WAVES) ? M2LC_WAVES / n_rt : 1, kmax = 2 * cols;
        kstep = (((kmax + want - 1) / want) + 15) & ~15;
        ns = want > 1 ? (kmax + kstep - 1) / kstep : 1;
    }
};

template <typename R, bool TRANS, int NT, int TAG>
__device__ __forceinline__ void chunk_block(int bid, int n_chunks, int s, int cols, int rmax,
                                            const int64_t *__restrict__ ch_mat, const int *__restrict__ ch_rank,
                                            const int *__restrict__ ch_pptr, const int64_t *__restrict__ pr_src,
                                            const int64_t *__restrict__ pr_pos,
                                            const typename Cx<R>::T *__restrict__ mat,
                                            const typename Cx<R>::T *__restrict__ in,
                                            typename Cx<R>::T *__restrict__ part)
{
    using C = typename Cx<R>::T;
    constexpr int PW = 16 * NT, PS = PW + 1;  // pairs per chunk, padded LDS row stride
    extern __shared__ unsigned char shraw[];
    R *XB = (R *)shraw;                        // [2 cols][PS]
    R *TB = XB + (size_t)2 * cols * PS;        // [2 rmax][PS]
    // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin, so XCD
    // x takes the contiguous chunk range [x per, (x + 1) per); chunks of one
    // operator are adjacent and reuse that XCD's L2
    const int per = (n_chunks + kXcds - 1) / kXcds;
    const int c = (bid % kXcds) * per + bid / kXcds;
    if (c >= n_chunks) return;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int p0 = ch_pptr[c], n = ch_pptr[c + 1] - p0;
    {
        // tpp threads per pair, each reading every tpp-th element of its pair's source vector
        constexpr int tpp = 64 * M2LC_WAVES / PW;
        const int p = tid / tpp, sub = tid - p * tpp;
        const bool pok = p < n;
        const C *src = in + (pok ? pr_src[p0 + p] : 0);
#pragma unroll 4
        for (int j = sub; j < cols; j += tpp) {
            const C v = src[j];
            XB[(2 * j) * PS + p] = pok ? v.x : (R)0;
            XB[(2 * j + 1) * PS + p] = pok ? v.y : (R)0;
        }
    }
    // scratch row of each of this lane's pairs (lane & 15 + 16 t), -1 past the chunk's end
    int64_t pos[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int p = 16 * t + (lane & 15);
        pos[t] = p < n ? pr_pos[p0 + p] : -1;
    }
    __syncthreads();
    const C *M = mat + ch_mat[c];
    const int r = ch_rank[c];
    R *P = (R *)part;
    auto to_part = [&](int row, int ci, int t, int, R v) {
        if (row < s && pos[t] >= 0) P[2 * (pos[t] * s + row) + ci] = v;
    };
    if (r < 0) {
        // dense s x cols, column-major (or its transpose stored cols x s)
        if (TRANS)
            mfma_rows<R, NT>(M, s, cols, (int64_t)cols, 1, XB, wv, lane, to_part);
        else
            mfma_rows<R, NT>(M, s, cols, 1, (int64_t)s, XB, wv, lane, to_part);
    } else {
        // T = V X (V: r x cols at M + s r, column-major), then Y = U T (U: s x r)
        const KSplit ks(r, cols);
        if (ks.ns == 1) {
            auto to_t = [&](int row, int ci, int, int p, R v) {
                if (row < r) TB[(2 * row + ci) * PS + p] = v;
            };
            mfma_rows<R, NT>(M + (size_t)s * r, r, cols, 1, (int64_t)r, XB, wv, lane, to_t);
            __syncthreads();
        } else {
            // slice q of T goes to rows [16 n_rt q, 16 n_rt (q + 1)) of TB, then slice 0 += 1, 2, 3
            const int q = wv / ks.n_rt, rt = wv - q * ks.n_rt, kb = q * ks.kstep;
            R *slab = TB + (size_t)q * 16 * ks.n_rt * PS;
            auto to_s = [&](int row, int ci, int, int p, R v) {
                if (row < r) slab[(2 * row + ci) * PS + p] = v;
            };
            if (q < ks.ns)
                mfma_tile<R, NT>(M + (size_t)s * r, r, 1, (int64_t)r, XB, rt, kb, min(2 * cols, kb + ks.kstep), lane,
                                 to_s);
            __syncthreads();
            const int stride = 16 * ks.n_rt * PS;
            for (int e = tid; e < 2 * r * PW; e += 64 * M2LC_WAVES) {
                const int row = e / PW, p = e - row * PW;
                R v = TB[row * PS + p];
                for (int j = 1; j < ks.ns; ++j) v += TB[j * stride + row * PS + p];
                TB[row * PS + p] = v;
            }
            __syncthreads();
        }
        mfma_rows<R, NT>(M, s, r, 1, (int64_t)s, TB, wv, lane, to_part);
    }
}

template <typename R, bool TRANS, int NT, int TAG>
__global__ __launch_bounds__(64 * M2LC_WAVES) void k_chunks_mfma(int n_chunks, int s, int cols, int rmax,
                                                                 const int64_t *__restrict__ ch_mat,
                                                                 const int *__restrict__ ch_rank,
                                                                 const int *__restrict__ ch_pptr,
                                                                 const int64_t *__restrict__ pr_src,
                                                                 const int64_t *__restrict__ pr_pos,
                                                                 const typename Cx<R>::T *__restrict__ mat,
                                                                 const typename Cx<R>::T *__restrict__ in,
                                                                 typename Cx<R>::T *__restrict__ part)
{
    chunk_block<R, TRANS, NT, TAG>(blockIdx.x, n_chunks, s, cols, rmax, ch_mat, ch_rank, ch_pptr, pr_src, pr_pos, mat,
                                   in, part);
}

// Sum of the per-pair results of each output slot (entries contiguous in
// target-major order), one wavefront per output, lanes over rows; four
// entries in flight per step, added in a fixed order.
template <typename R>
__device__ __forceinline__ void seg_sum_block(int bid, int n_out, int s, const int64_t *__restrict__ red_out,
                                              const int64_t *__restrict__ red_ptr,
                                              const typename Cx<R>::T *__restrict__ part, typename Cx<R>::T *out)
{
    using C = typename Cx<R>::T;
    const int o = bid * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (o >= n_out) return;
    const int64_t e0 = red_ptr[o], e1 = red_ptr[o + 1];
    C *dst = out + red_out[o];
    for (int row = lane; row < s; row += 64) {
        C a0 = Cx<R>::mk(0, 0), a1 = a0, a2 = a0, a3 = a0;
        const C *pp = part + e0 * s + row;
        int64_t e = e0;
        for (; e + 4 <= e1; e += 4, pp += 4 * (int64_t)s) {
            const C v0 = pp[0], v1 = pp[s], v2 = pp[2 * (int64_t)s], v3 = pp[3 * (int64_t)s];
            a0 = cadd(a0, v0);
            a1 = cadd(a1, v1);
            a2 = cadd(a2, v2);
            a3 = cadd(a3, v3);
        }
        for (; e < e1; ++e, pp += s) a0 = cadd(a0, pp[0]);
        dst[row] = cadd(dst[row], cadd(cadd(a0, a1), cadd(a2, a3)));
    }
}

template <typename R, int TAG>
__global__ __launch_bounds__(256) void k_seg_sum(int n_out, int s, const int64_t *__restrict__ red_out,
                                                 const int64_t *__restrict__ red_ptr,
                                                 const typename Cx<R>::T *__restrict__ part,
                                                 typename Cx<R>::T *out)
{
    seg_sum_block<R>(blockIdx.x, n_out, s, red_out, red_ptr, part, out);
}

// One launch for two slabs of the partial-sum schedule: the first n_seg
// workgroups sum the per-pair results of the previous slab (scratch buffer
// prev) into its outputs while the others run the current slab's chunks into
// the other scratch buffer, so the bandwidth-bound sums overlap the
// latency-bound chunks and the launch tails.  n_seg is a multiple of the XCD
// count, so the chunk workgroups keep their XCD-aware order.
template <typename R, bool TRANS, int NT, int TAG>
__global__ __launch_bounds__(64 * M2LC_WAVES) void k_chunks_seg(
    int n_seg, int n_out_prev, int s_prev, const int64_t *__restrict__ red_out_prev,
    const int64_t *__restrict__ red_ptr_prev, const typename Cx<R>::T *__restrict__ prev,
    typename Cx<R>::T *out_prev, int n_chunks, int s, int cols, int rmax, const int64_t *__restrict__ ch_mat,
    const int *__restrict__ ch_rank, const int *__restrict__ ch_pptr, const int64_t *__restrict__ pr_src,
    const int64_t *__restrict__ pr_pos, const typename Cx<R>::T *__restrict__ mat,
    const typename Cx<R>::T *__restrict__ in, typename Cx<R>::T *__restrict__ part)
{
    if ((int)blockIdx.x < n_seg) {
        seg_sum_block<R>(blockIdx.x, n_out_prev, s_prev, red_out_prev, red_ptr_prev, prev, out_prev);
        return;
    }
    chunk_block<R, TRANS, NT, TAG>(blockIdx.x - n_seg, n_chunks, s, cols, rmax, ch_mat, ch_rank, ch_pptr, pr_src,
                                   pr_pos, mat, in, part);
}

// Translation chunks, one wavefront per chunk of <= 16 pairs sharing one
// operator (four chunks per workgroup): no LDS and no barrier.  The operator
// comes from a row-major copy of the pool: dense A (s x cols), or U (s x r)
// followed by V (r x cols) of a low-rank one.  Real inner index k of four
// consecutive matrix-core steps (g, t) is 16 g + 4 k4 + t for lane group k4,
// so that a lane reads two adjacent complex entries of an operator row or of
// its source vector per four steps.  The A row that each lane supplies is
// permuted by Mf::rho, so that result register q of lane group k4 holds real
// row 4 k4 + q of the tile: for a low-rank operator the result T = V X is then
// already the B operand of Y = U T (register q of T tile g is step (g, q)),
// and a lane stores two adjacent complex rows of Y.
constexpr int WV_GMAX = 8;   // dense operators of at most 64 columns hold the sources in registers
constexpr int WV_RMAX = 32;  // low-rank operators: rank at most 32

// Four A values of lane row I (real row of the product) at the inner group
// starting at complex column j0: entries (i, j0) and (i, j0 + 1) of the
// row-major complex matrix M (nrow x ncol), zero outside it.
template <typename R>
__device__ __forceinline__ void wv_a(const typename Cx<R>::T *__restrict__ M, int nrow, int ncol, int I, int j0,
                                     R a[4])
{
    using C = typename Cx<R>::T;
    const int i = I >> 1;
    const bool im = I & 1, rok = i < nrow, ok0 = rok && j0 < ncol, ok1 = rok && j0 + 1 < ncol;
    const C *p = M + (int64_t)(rok ? i : 0) * ncol;
    const C m0 = p[ok0 ? j0 : 0], m1 = p[ok1 ? j0 + 1 : 0];
    const R r0 = ok0 ? m0.x : (R)0, i0 = ok0 ? m0.y : (R)0, r1 = ok1 ? m1.x : (R)0, i1 = ok1 ? m1.y : (R)0;
    // row (Re, Im) of y_i against inner (Re, Im) of x_j: [Re -Im; Im Re]
    a[0] = im ? i0 : r0;
    a[1] = im ? r0 : -i0;
    a[2] = im ? i1 : r1;
    a[3] = im ? r1 : -i1;
}

// Four B values: (Re, Im) of entries j0 and j0 + 1 of a source vector
template <typename R>
__device__ __forceinline__ void wv_b(const typename Cx<R>::T *__restrict__ x, int ncol, int j0, bool pok, R b[4])
{
    using C = typename Cx<R>::T;
    const bool ok0 = pok && j0 < ncol, ok1 = pok && j0 + 1 < ncol;
    const C x0 = x[ok0 ? j0 : 0], x1 = x[ok1 ? j0 + 1 : 0];
    b[0] = ok0 ? x0.x : (R)0;
    b[1] = ok0 ? x0.y : (R)0;
    b[2] = ok1 ? x1.x : (R)0;
    b[3] = ok1 ? x1.y : (R)0;
}

// Complex rows 8 rt + 2 k4 and the next of a result tile to the pair's scratch row
template <typename R>
__device__ __forceinline__ void wv_store(typename Cx<R>::T *dst, bool ok, int s, int rt, int k4,
                                         const typename Mf<R>::V &y)
{
    const int m0 = 8 * rt + 2 * k4;
    if (ok && m0 < s) dst[m0] = Cx<R>::mk(y[0], y[1]);
    if (ok && m0 + 1 < s) dst[m0 + 1] = Cx<R>::mk(y[2], y[3]);
}

// Y = A X for a dense operator, cols <= 64: the source groups stay in
// registers and the row tiles go two at a time (two independent chains)
template <typename R>
__device__ __forceinline__ void wv_dense(const typename Cx<R>::T *__restrict__ A, int s, int cols,
                                         const typename Cx<R>::T *__restrict__ x, bool pok,
                                         typename Cx<R>::T *dst, int i16, int k4)
{
    typedef typename Mf<R>::V V;
    const int G = (2 * cols + 15) >> 4, n_rt = (2 * s + 15) >> 4, rw = Mf<R>::rho(i16);
    R xb[WV_GMAX][4];
#pragma unroll
    for (int g = 0; g < WV_GMAX; ++g) {
        if (g < G) {
            wv_b<R>(x, cols, 8 * g + 2 * k4, pok, xb[g]);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) xb[g][t] = (R)0;
        }
    }
    int rt = 0;
    for (; rt + 1 < n_rt; rt += 2) {
        V y0 = {0, 0, 0, 0}, y1 = y0;
#pragma unroll
        for (int g = 0; g < WV_GMAX; ++g) {
            if (g < G) {
                R a0[4], a1[4];
                wv_a<R>(A, s, cols, 16 * rt + rw, 8 * g + 2 * k4, a0);
                wv_a<R>(A, s, cols, 16 * rt + 16 + rw, 8 * g + 2 * k4, a1);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    y0 = Mf<R>::mma(a0[t], xb[g][t], y0);
                    y1 = Mf<R>::mma(a1[t], xb[g][t], y1);
                }
            }
        }
        wv_store<R>(dst, pok, s, rt, k4, y0);
        wv_store<R>(dst, pok, s, rt + 1, k4, y1);
    }
    if (rt < n_rt) {
        V y0 = {0, 0, 0, 0};
#pragma unroll
        for (int g = 0; g < WV_GMAX; ++g) {
            if (g < G) {
                R a0[4];
                wv_a<R>(A, s, cols, 16 * rt + rw, 8 * g + 2 * k4, a0);
#pragma unroll
                for (int t = 0; t < 4; ++t) y0 = Mf<R>::mma(a0[t], xb[g][t], y0);
            }
        }
        wv_store<R>(dst, pok, s, rt, k4, y0);
    }
}

// Y = A X for a dense operator of any width on NP tiles of 16 pairs: the
// source groups are read again for every pair of row tiles (same products
// in the same order as wv_dense, so the same result bit for bit)
template <typename R, int NP>
__device__ __forceinline__ void wv_dense_stream(const typename Cx<R>::T *__restrict__ A, int s, int cols,
                                                const typename Cx<R>::T *const x[NP], const bool pok[NP],
                                                typename Cx<R>::T *const dst[NP], int i16, int k4)
{
    typedef typename Mf<R>::V V;
    const int G = (2 * cols + 15) >> 4, n_rt = (2 * s + 15) >> 4, rw = Mf<R>::rho(i16);
    int rt = 0;
    for (; rt + 1 < n_rt; rt += 2) {
        V y0[NP], y1[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) y0[p] = y1[p] = V{0, 0, 0, 0};
        for (int g = 0; g < G; ++g) {
            R a0[4], a1[4], xb[NP][4];
#pragma unroll
            for (int p = 0; p < NP; ++p) wv_b<R>(x[p], cols, 8 * g + 2 * k4, pok[p], xb[p]);
            wv_a<R>(A, s, cols, 16 * rt + rw, 8 * g + 2 * k4, a0);
            wv_a<R>(A, s, cols, 16 * rt + 16 + rw, 8 * g + 2 * k4, a1);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    y0[p] = Mf<R>::mma(a0[t], xb[p][t], y0[p]);
                    y1[p] = Mf<R>::mma(a1[t], xb[p][t], y1[p]);
                }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            wv_store<R>(dst[p], pok[p], s, rt, k4, y0[p]);
            wv_store<R>(dst[p], pok[p], s, rt + 1, k4, y1[p]);
        }
    }
    if (rt < n_rt) {
        V y0[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) y0[p] = V{0, 0, 0, 0};
        for (int g = 0; g < G; ++g) {
            R a0[4], xb[NP][4];
#pragma unroll
            for (int p = 0; p < NP; ++p) wv_b<R>(x[p], cols, 8 * g + 2 * k4, pok[p], xb[p]);
            wv_a<R>(A, s, cols, 16 * rt + rw, 8 * g + 2 * k4, a0);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int p = 0; p < NP; ++p) y0[p] = Mf<R>::mma(a0[t], xb[p][t], y0[p]);
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) wv_store<R>(dst[p], pok[p], s, rt, k4, y0[p]);
    }
}

// Y = U (V X) for a low-rank operator with 2 r <= 16 RT rows of T, on NP
// tiles of 16 pairs (every operator value loaded feeds NP products; a pair's
// result does not depend on NP bit for bit)
template <typename R, int RT, int NP>
__device__ __forceinline__ void wv_lowrank(const typename Cx<R>::T *__restrict__ M, int s, int cols, int r,
                                           const typename Cx<R>::T *const x[NP], const bool pok[NP],
                                           typename Cx<R>::T *const dst[NP], int i16, int k4)
{
    typedef typename Mf<R>::V V;
    const typename Cx<R>::T *U = M, *Vm = M + (int64_t)s * r;
    const int G = (2 * cols + 15) >> 4, n_rt = (2 * s + 15) >> 4, rw = Mf<R>::rho(i16);
    // T = V X; with one tile of T, even and odd inner groups go to two
    // partial sums (independent chains), added in a fixed order at the end
    constexpr bool two = RT == 1;
    V t[RT][NP], t2[RT][NP];
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
        for (int p = 0; p < NP; ++p) t[q][p] = t2[q][p] = V{0, 0, 0, 0};
    int g = 0;
    for (; g + 1 < G; g += 2) {
        R b0[NP][4], b1[NP][4];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            wv_b<R>(x[p], cols, 8 * g + 2 * k4, pok[p], b0[p]);
            wv_b<R>(x[p], cols, 8 * g + 8 + 2 * k4, pok[p], b1[p]);
        }
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            R a0[4], a1[4];
            wv_a<R>(Vm, r, cols, 16 * q + rw, 8 * g + 2 * k4, a0);
            wv_a<R>(Vm, r, cols, 16 * q + rw, 8 * g + 8 + 2 * k4, a1);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int p = 0; p < NP; ++p) t[q][p] = Mf<R>::mma(a0[u], b0[p][u], t[q][p]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if (two)
                        t2[q][p] = Mf<R>::mma(a1[u], b1[p][u], t2[q][p]);
                    else
                        t[q][p] = Mf<R>::mma(a1[u], b1[p][u], t[q][p]);
                }
        }
    }
    if (g < G) {
        R b0[NP][4];
#pragma unroll
        for (int p = 0; p < NP; ++p) wv_b<R>(x[p], cols, 8 * g + 2 * k4, pok[p], b0[p]);
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            R a0[4];
            wv_a<R>(Vm, r, cols, 16 * q + rw, 8 * g + 2 * k4, a0);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int p = 0; p < NP; ++p) t[q][p] = Mf<R>::mma(a0[u], b0[p][u], t[q][p]);
        }
    }
    if (two) {
#pragma unroll
        for (int q = 0; q < RT; ++q)
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int e = 0; e < 4; ++e) t[q][p][e] += t2[q][p][e];
    }
    // Y = U T, two row tiles at a time
    int rt = 0;
    for (; rt + 1 < n_rt; rt += 2) {
        V y0[NP], y1[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) y0[p] = y1[p] = V{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            R a0[4], a1[4];
            wv_a<R>(U, s, r, 16 * rt + rw, 8 * q + 2 * k4, a0);
            wv_a<R>(U, s, r, 16 * rt + 16 + rw, 8 * q + 2 * k4, a1);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    y0[p] = Mf<R>::mma(a0[u], t[q][p][u], y0[p]);
                    y1[p] = Mf<R>::mma(a1[u], t[q][p][u], y1[p]);
                }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            wv_store<R>(dst[p], pok[p], s, rt, k4, y0[p]);
            wv_store<R>(dst[p], pok[p], s, rt + 1, k4, y1[p]);
        }
    }
    if (rt < n_rt) {
        V y0[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) y0[p] = V{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            R a0[4];
            wv_a<R>(U, s, r, 16 * rt + rw, 8 * q + 2 * k4, a0);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int p = 0; p < NP; ++p) y0[p] = Mf<R>::mma(a0[u], t[q][p][u], y0[p]);
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) wv_store<R>(dst[p], pok[p], s, rt, k4, y0[p]);
    }
}

// One launch of the wavefront chunks, the first n_seg workgroups summing the
// previous slab's per-pair results as in k_chunks_seg (n_seg = 0: none).
// Chunk workgroups are dealt to the XCDs in contiguous ranges.  KIND names
// the operators a slab holds, so that an instance keeps only the registers
// its paths need: 0 dense, 1 low-rank of rank <= 16, 2 low-rank, 3 both, 4
// both with the dense sources read per row-tile pair (any width), 5 dense
// read so.
// NP: tiles of 16 pairs per chunk (2 not with kinds 0 and 3).
template <typename R, int TAG, int KIND, int NP>
__global__ __launch_bounds__(256) void k_wave_seg(
    int n_seg, int n_out_prev, int s_prev, const int64_t *__restrict__ red_out_prev,
    const int64_t *__restrict__ red_ptr_prev, const typename Cx<R>::T *__restrict__ prev,
    typename Cx<R>::T *out_prev, int n_chunks, int s, int cols, const int64_t *__restrict__ ch_mat,
    const int *__restrict__ ch_rank, const int *__restrict__ ch_pptr, const int64_t *__restrict__ pr_src,
    const int64_t *__restrict__ pr_pos, const typename Cx<R>::T *__restrict__ mat,
    const typename Cx<R>::T *__restrict__ in, typename Cx<R>::T *__restrict__ part)
{
    using C = typename Cx<R>::T;
    static_assert(NP == 1 || (KIND != 0 && KIND != 3), "two pair tiles need the streaming dense path");
    if ((int)blockIdx.x < n_seg) {
        seg_sum_block<R>(blockIdx.x, n_out_prev, s_prev, red_out_prev, red_ptr_prev, prev, out_prev);
        return;
    }
    const int b = (int)blockIdx.x - n_seg, nb = (n_chunks + 3) >> 2, per = (nb + kXcds - 1) / kXcds;
    const int c = 4 * ((b % kXcds) * per + b / kXcds) + (int)(threadIdx.x >> 6);
    if (c >= n_chunks) return;
    const int lane = threadIdx.x & 63, i16 = lane & 15, k4 = lane >> 4;
    const int p0 = ch_pptr[c], n = ch_pptr[c + 1] - p0;
    bool pok[NP];
    const C *x[NP];
    C *dst[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int e = i16 + 16 * p;
        pok[p] = e < n;
        x[p] = in + (pok[p] ? pr_src[p0 + e] : 0);
        dst[p] = part + (pok[p] ? pr_pos[p0 + e] : 0) * (int64_t)s;
    }
    const C *M = mat + ch_mat[c];
    const int r = ch_rank[c];
    if constexpr (KIND == 0) {
        wv_dense<R>(M, s, cols, x[0], pok[0], dst[0], i16, k4);
    } else if constexpr (KIND == 5) {
        wv_dense_stream<R, NP>(M, s, cols, x, pok, dst, i16, k4);
    } else if constexpr (KIND == 3) {
        if (r < 0)
            wv_dense<R>(M, s, cols, x[0], pok[0], dst[0], i16, k4);
        else if (r <= 8)
            wv_lowrank<R, 1, 1>(M, s, cols, r, x, pok, dst, i16, k4);
        else if (r <= 16)
            wv_lowrank<R, 2, 1>(M, s, cols, r, x, pok, dst, i16, k4);
        else if (r <= 24)
            wv_lowrank<R, 3, 1>(M, s, cols, r, x, pok, dst, i16, k4);
        else
            wv_lowrank<R, 4, 1>(M, s, cols, r, x, pok, dst, i16, k4);
    } else if constexpr (KIND == 4) {
        if (r < 0)
            wv_dense_stream<R, NP>(M, s, cols, x, pok, dst, i16, k4);
        else if (r <= 8)
            wv_lowrank<R, 1, NP>(M, s, cols, r, x, pok, dst, i16, k4);
        else if (r <= 16)
            wv_lowrank<R, 2, NP>(M, s, cols, r, x, pok, dst, i16, k4);
        else if (r <= 24)
            wv_lowrank<R, 3, NP>(M, s, cols, r, x, pok, dst, i16, k4);
        else
            wv_lowrank<R, 4, NP>(M, s, cols, r, x, pok, dst, i16, k4);
    } else {
        if (r <= 8)
            wv_lowrank<R, 1, NP>(M, s, cols, r, x, pok, dst, i16, k4);
        else if (KIND == 1 || r <= 16)
            wv_lowrank<R, 2, NP>(M, s, cols, r, x, pok, dst, i16, k4);
        else if (r <= 24)
            wv_lowrank<R, 3, NP>(M, s, cols, r, x, pok, dst, i16, k4);
        else
            wv_lowrank<R, 4, NP>(M, s, cols, r, x, pok, dst, i16, k4);
    }
}

template <typename R, int TAG>
static void launch_wave(const DChunks &c, dim3 grid, hipStream_t st, int n_seg, int n_out_prev, int s_prev,
                        const int64_t *ro, const int64_t *rp, const typename Cx<R>::T *prev,
                        typename Cx<R>::T *out_prev, const typename Cx<R>::T *mw, const typename Cx<R>::T *in,
                        typename Cx<R>::T *part)
{
#define FDBEM_WAVE(K, NP)                                                                                            \
    hipLaunchKernelGGL((k_wave_seg<R, TAG, K, NP>), grid, dim3(256), 0, st, n_seg, n_out_prev, s_prev, ro, rp,     \
                       prev, out_prev, c.n, c.s, c.cols, c.ch_matw, c.ch_rank, c.ch_pptr, c.pr_src, c.pr_pos, mw, in, \
                       part)
    const bool two = c.pw == 32;
    switch (c.wave_kind) {
    case 0: FDBEM_WAVE(0, 1); break;
    case 1: if (two) FDBEM_WAVE(1, 2); else FDBEM_WAVE(1, 1); break;
    case 2: if (two) FDBEM_WAVE(2, 2); else FDBEM_WAVE(2, 1); break;
    case 3: FDBEM_WAVE(3, 1); break;
    case 4: if (two) FDBEM_WAVE(4, 2); else FDBEM_WAVE(4, 1); break;
    default: if (two) FDBEM_WAVE(5, 2); else FDBEM_WAVE(5, 1); break;
    }
#undef FDBEM_WAVE
}

__global__ void k_corr(const int64_t *__restrict__ rp, const int32_t *__restrict__ blk,
                       const double2 *__restrict__ val, const double2 *__restrict__ in, double2 *__restrict__ out,
                       int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t b = rp[i]; b < rp[i + 1]; ++b) {
        const double2 *u = in + 6 * (int64_t)blk[b];
        const double2 *v = val + 6 * b;
#pragma unroll
        for (int g = 0; g < 6; ++g) acc = cadd(acc, cmul(v[g], u[g]));
    }
    out[i] = cadd(out[i], acc);
}

__global__ void k_plane_wave(const double *__restrict__ X, const double *__restrict__ Y, const double *__restrict__ Z,
                             const double *__restrict__ NX, const double *__restrict__ NY, const double *__restrict__ NZ,
                             const int64_t *__restrict__ perm, double k, double coupling, double d0, double d1,
                             double d2, double2 *__restrict__ rhs, int64_t n)
{
    // b = u_inc + alpha du_inc/dn_x, u_inc = exp(ik x.d), du_inc/dn = ik (d.n) u_inc, alpha = i c/k
    // => b = u_inc (1 + (i c/k)(ik)(d.n)) = u_inc (1 - c d.n)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sn, cs;
    sincos(k * (X[i] * d0 + Y[i] * d1 + Z[i] * d2), &sn, &cs);
    const double f = 1.0 - coupling * (NX[i] * d0 + NY[i] * d1 + NZ[i] * d2);
    rhs[perm[i]] = make_double2(cs * f, sn * f);
}

// Neumann data on the right-hand side: rhs_i -= a q_i with a = alpha c the
// jump term of the adjoint operator (c = 1/2 on a smooth surface).
__global__ void k_sub_scaled(const double2 *__restrict__ q, double a_re, double a_im, double2 *__restrict__ rhs,
                             int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 v = q[i];
    double2 r = rhs[i];
    r.x -= a_re * v.x - a_im * v.y;
    r.y -= a_re * v.y + a_im * v.x;
    rhs[i] = r;
}

// ---------------------------------------------------------------- host side
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
static T *dalloc(Device &D, size_t n)
{
    if (n == 0) n = 1;
    void *p = nullptr;
    HIP_CHECK(hipMalloc(&p, n * sizeof(T)));
    D.allocs.push_back(p);
    D.bytes += n * sizeof(T);
    return (T *)p;
}

template <typename T>
static T *dupload(Device &D, const std::vector<T> &v)
{
    T *p = dalloc<T>(D, v.size());
    if (!v.empty()) HIP_CHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

static DGemv upload_gemv(Device &D, const GemvList &G)
{
    DGemv g;
    g.n_out = (int)G.out_off.size();
    g.rows = G.rows;
    g.cols = G.cols;
    g.trans = G.trans;
    g.n_ent = (int64_t)G.in_off.size();
    if (g.n_out == 0) return g;
    g.out_off = dupload(D, G.out_off);
    g.ptr = dupload(D, G.ptr);
    g.in_off = dupload(D, G.in_off);
    g.mat_off = dupload(D, G.mat_off);
    g.rank = dupload(D, G.rank);
    for (int r : G.rank) g.max_rank = std::max(g.max_rank, r);
    if (g.rows > GEMV_MAXROWS) throw std::runtime_error("reduced dimension exceeds the GEMV kernel's limit");
    return g;
}

static DTiles upload_tiles(Device &D, const M2LTiles &T)
{
    DTiles d;
    d.n_tiles = (int)T.tile_ntgt.size();
    d.s = T.s;
    d.rmax = std::max(1, T.max_rank);
    d.tile = T.tile;
    d.chunk = T.chunk;
    if (d.n_tiles == 0) return d;
    d.shm = sizeof(double2) * ((size_t)(d.tile + d.chunk) * d.s + (size_t)d.chunk * d.rmax);
    d.tgt_off = dupload(D, T.tgt_off);
    d.tile_ntgt = dupload(D, T.tile_ntgt);
    d.tile_cptr = dupload(D, T.tile_cptr);
    d.ch_mat = dupload(D, T.ch_mat);
    d.ch_rank = dupload(D, T.ch_rank);
    d.ch_pptr = dupload(D, T.ch_pptr);
    d.pr_tl = dupload(D, T.pr_tl);
    d.pr_src = dupload(D, T.pr_src);
    return d;
}

// pairs per slab: the scratch of per-pair results stays within slab_mb MiB
static int64_t slab_entries(const GemvList &G, int slab_mb)
{
    return std::max<int64_t>(1, ((int64_t)slab_mb << 20) / (16 * std::max(1, G.rows)));
}

// LDS of the chunk kernel: sources [2 cols][pw + 1] and T [tb rows][pw + 1];
// low-rank chunks need at least 64 rows of T for the split first product
static size_t mfma_shm(const DChunks &c)
{
    const size_t tb = (size_t)(c.lowrank ? std::max(2 * c.rmax, 64) : 2 * c.rmax);
    return sizeof(double) * (c.pw + 1) * (2 * (size_t)c.cols + tb);
}

static DChunks upload_chunks(Device &D, const M2LChunks &C)
{
    DChunks d;
    d.n = (int)C.ch_mat.size();
    d.s = C.s;
    d.cols = C.cols;
    d.rmax = std::max(1, C.max_rank);
    d.lowrank = C.max_rank > 0;
    if (d.n == 0) return d;
    d.shm = sizeof(double2) * (size_t)M2LC_WAVES * (M2LC_CH * d.cols + M2LC_CH * d.rmax);
    d.ch_mat = dupload(D, C.ch_mat);
    d.ch_rank = dupload(D, C.ch_rank);
    d.ch_pptr = dupload(D, C.ch_pptr);
    d.pr_tgt = dupload(D, C.pr_tgt);
    d.pr_src = dupload(D, C.pr_src);
    d.pw = C.chunk;
    if (!C.red_out.empty()) {
        d.n_out = (int)C.red_out.size();
        d.n_entries = (int64_t)C.pr_pos.size();
        d.pr_pos = dupload(D, C.pr_pos);
        d.red_out = dupload(D, C.red_out);
        d.red_ptr = dupload(D, C.red_ptr);
    }
    return d;
}

// Row-major copies of a slab's operators for the wavefront chunk kernel,
// shared by every slab that uses them (key: pool offset and transposed use).
// Returns the per-chunk offsets into `pool`, or an empty vector when some
// operator does not fit the kernel (a rank above 32); with pool == nullptr
// every operator must already be there.
static std::vector<int64_t> wave_offsets(const Plan &P, const M2LChunks &C,
                                         std::unordered_map<int64_t, int64_t> &map, std::vector<double2> *pool)
{
    std::vector<int64_t> off(C.ch_mat.size());
    for (size_t q = 0; q < C.ch_mat.size(); ++q) {
        const int r = C.ch_rank[q];
        if (r > WV_RMAX) return {};
    }
    const int s = C.s, cols = C.cols;
    for (size_t q = 0; q < C.ch_mat.size(); ++q) {
        const int r = C.ch_rank[q];
        const int64_t key = 2 * C.ch_mat[q] + (C.trans ? 1 : 0);
        auto it = map.find(key);
        if (it != map.end()) {
            off[q] = it->second;
            continue;
        }
        if (!pool) throw std::runtime_error("translation operator missing from the wavefront pool");
        const int64_t o = (int64_t)pool->size();
        const cplx *M = P.matpool.data() + C.ch_mat[q];
        auto put = [&](const cplx &v) { pool->push_back(make_double2(v.real(), v.imag())); };
        if (r < 0) {
            // A (s x cols): the pool holds A column-major, or its transpose for the transposed use
            for (int i = 0; i < s; ++i)
                for (int j = 0; j < cols; ++j) put(C.trans ? M[(int64_t)i * cols + j] : M[i + (int64_t)j * s]);
        } else {
            // U (s x r) at M and V (r x cols) at M + s r, both column-major in the pool
            for (int i = 0; i < s; ++i)
                for (int m = 0; m < r; ++m) put(M[i + (int64_t)m * s]);
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < cols; ++j) put(M[(int64_t)s * r + i + (int64_t)j * r]);
        }
        map.emplace(key, o);
        off[q] = o;
    }
    return off;
}

// Whether every operator of a translation list fits the wavefront kernel
static bool wave_fits(const GemvList &G)
{
    for (int r : G.rank)
        if (r > WV_RMAX) return false;
    return true;
}

// Put a slab on the wavefront kernel when all its operators fit it: offsets
// into the row-major pool (added to `pool`, or looked up once the pool is on
// the device: pool == nullptr) and the kind of operators it holds.
static void attach_wave(Device &D, const Plan &P, const M2LChunks &C, DChunks &d, std::vector<double2> *pool)
{
    bool dense = false, low = false;
    int rmax = 0;
    for (int r : C.ch_rank) {
        (r < 0 ? dense : low) = true;
        rmax = std::max(rmax, r);
    }
    const std::vector<int64_t> off = wave_offsets(P, C, D.wmap, pool);
    if (off.empty()) return;
    d.ch_matw = dupload(D, off);
    // dense operators on 32-pair chunks, or wider than 64 columns, take the streaming dense path
    const bool stream = C.cols > 8 * WV_GMAX || C.chunk > M2LC_CH;
    d.wave_kind = !low ? (stream ? 5 : 0) : !dense ? (rmax <= 16 ? 1 : 2) : stream ? 4 : 3;
    d.matw = D.matw;
    d.matwf = D.matwf;
}

static DLeaf upload_leaf(Device &D, const Plan &P, const std::vector<LeafTask> &T)
{
    DLeaf L;
    L.n = (int)T.size();
    if (L.n == 0) return L;
    std::vector<int64_t> s(L.n), e(L.n), sl(L.n);
    std::vector<int> tm(L.n);
    std::vector<double> c(3 * L.n);
    for (int i = 0; i < L.n; ++i) {
        s[i] = T[i].start;
        e[i] = T[i].end;
        sl[i] = T[i].slot_off;
        tm[i] = T[i].tmpl;
        c[3 * i] = T[i].center[0];
        c[3 * i + 1] = T[i].center[1];
        c[3 * i + 2] = T[i].center[2];
    }
    std::vector<int> gp{0};
    for (int i = 1; i <= L.n; ++i)
        if (i == L.n || tm[i] != tm[gp.back()] || i - gp.back() == L2T_G) gp.push_back(i);
    L.n_groups = (int)gp.size() - 1;
    L.gptr = dupload(D, gp);
    L.start = dupload(D, s);
    L.end = dupload(D, e);
    L.slot = dupload(D, sl);
    L.tmpl = dupload(D, tm);
    L.center = dupload(D, c);
    return L;
}

template <int TAG, bool TRANS, typename R>
static void launch_slabs(const std::vector<DChunks> &S, void *part, const typename Cx<R>::T *mat,
                         const typename Cx<R>::T *in, typename Cx<R>::T *out, hipStream_t st);

static void free_chunks(Device &D, DChunks &c)
{
    for (void *p : {(void *)c.ch_mat, (void *)c.pr_tgt, (void *)c.pr_src, (void *)c.ch_rank, (void *)c.ch_pptr,
                    (void *)c.pr_pos, (void *)c.red_out, (void *)c.red_ptr, (void *)c.ch_matw}) {
        if (!p) continue;
        auto it = std::find(D.allocs.begin(), D.allocs.end(), p);
        if (it != D.allocs.end()) D.allocs.erase(it);
        (void)hipFree(p);
    }
    c = DChunks();
}

// Dynamic LDS limit of every matrix-core chunk kernel instance, raised to at
// least `bytes` (the default limit is 64 KiB).  The attribute belongs to the
// kernel on the device, not to a plan, so the limit reached on each device is
// kept process-wide and only ever raised: a later plan with smaller chunks
// must not lower it below what an earlier plan's launches need.
static void set_mfma_lds(Device &D, size_t bytes)
{
    static std::mutex mu;
    static std::map<int, size_t> reached;  // device -> limit set so far
    std::lock_guard<std::mutex> lock(mu);
    size_t &have = reached[D.device];
    D.mfma_lds = std::max(D.mfma_lds, have);
    if (bytes <= 65536 || bytes <= have) return;
    for (const void *f : {(const void *)k_chunks_mfma<double, false, 1, TAG_M2L>,
                          (const void *)k_chunks_mfma<double, false, 1, TAG_M2M>,
                          (const void *)k_chunks_mfma<double, true, 1, TAG_L2L>,
                          (const void *)k_chunks_mfma<float, false, 1, TAG_M2L>,
                          (const void *)k_chunks_mfma<float, false, 1, TAG_M2M>,
                          (const void *)k_chunks_mfma<float, true, 1, TAG_L2L>,
                          (const void *)k_chunks_mfma<double, false, 2, TAG_M2L>,
                          (const void *)k_chunks_mfma<double, false, 2, TAG_M2M>,
                          (const void *)k_chunks_mfma<double, true, 2, TAG_L2L>,
                          (const void *)k_chunks_mfma<float, false, 2, TAG_M2L>,
                          (const void *)k_chunks_mfma<float, false, 2, TAG_M2M>,
                          (const void *)k_chunks_mfma<float, true, 2, TAG_L2L>,
                          (const void *)k_chunks_seg<double, false, 1, TAG_M2L>,
                          (const void *)k_chunks_seg<double, false, 1, TAG_M2M>,
                          (const void *)k_chunks_seg<double, true, 1, TAG_L2L>,
                          (const void *)k_chunks_seg<float, false, 1, TAG_M2L>,
                          (const void *)k_chunks_seg<float, false, 1, TAG_M2M>,
                          (const void *)k_chunks_seg<float, true, 1, TAG_L2L>,
                          (const void *)k_chunks_seg<double, false, 2, TAG_M2L>,
                          (const void *)k_chunks_seg<double, false, 2, TAG_M2M>,
                          (const void *)k_chunks_seg<double, true, 2, TAG_L2L>,
                          (const void *)k_chunks_seg<float, false, 2, TAG_M2L>,
                          (const void *)k_chunks_seg<float, false, 2, TAG_M2M>,
                          (const void *)k_chunks_seg<float, true, 2, TAG_L2L>})
        HIP_CHECK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    have = bytes;
    D.mfma_lds = bytes;
}

// Builder autotuner: for every M2L level, time the matrix-core chunk kernel
// with 16 and with 32 pairs per chunk (one or two pair tiles per operator
// element loaded) on this plan's own lists and keep the faster.  Both shapes
// give bitwise the same result.
static void autotune_m2l(Plan &P, Device &D)
{
    const bool f32 = D.prec == 1;
    if (f32) {
        hipLaunchKernelGGL(k_fill_zero<float2>, dim3(nblk(D.n_od, 256)), dim3(256), 0, 0, D.odf, D.n_od);
        hipLaunchKernelGGL(k_fill_zero<float2>, dim3(nblk(D.n_id, 256)), dim3(256), 0, 0, D.idf, D.n_id);
    } else {
        hipLaunchKernelGGL(k_fill_zero<double2>, dim3(nblk(D.n_od, 256)), dim3(256), 0, 0, D.od, D.n_od);
        hipLaunchKernelGGL(k_fill_zero<double2>, dim3(nblk(D.n_id, 256)), dim3(256), 0, 0, D.id, D.n_id);
    }
    int maxsh = 65536;
    (void)hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, D.device);
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    // kind 0: M2L (od -> id), 1: M2M (od -> od), 2: L2L (id -> id, transposed operators)
    auto launch = [&](int kind, const std::vector<DChunks> &S) {
        if (f32) {
            if (kind == 0) launch_slabs<TAG_M2L, false, float>(S, D.part, D.matf, D.odf, D.idf, 0);
            if (kind == 1) launch_slabs<TAG_M2M, false, float>(S, D.part, D.matf, D.odf, D.odf, 0);
            if (kind == 2) launch_slabs<TAG_L2L, true, float>(S, D.part, D.matf, D.idf, D.idf, 0);
        } else {
            if (kind == 0) launch_slabs<TAG_M2L, false, double>(S, D.part, D.mat, D.od, D.id, 0);
            if (kind == 1) launch_slabs<TAG_M2M, false, double>(S, D.part, D.mat, D.od, D.od, 0);
            if (kind == 2) launch_slabs<TAG_L2L, true, double>(S, D.part, D.mat, D.id, D.id, 0);
        }
    };
    auto time = [&](int kind, const std::vector<DChunks> &S) {
        float best = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
            HIP_CHECK(hipEventRecord(e0, 0));
            launch(kind, S);
            HIP_CHECK(hipEventRecord(e1, 0));
            HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0;
            HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) best = std::min(best, ms);
        }
        return (double)best;
    };
    static const char *names[3] = {"M2L", "M2M", "L2L"};
    for (int kind = 0; kind < 3; ++kind) {
        std::vector<std::vector<DChunks>> &slabs = kind == 0 ? D.m2ls : kind == 1 ? D.m2ms : D.l2ls;
        const std::vector<GemvList> &lists = kind == 0 ? P.m2l_lists : kind == 1 ? P.m2m_lists : P.l2l_lists;
        for (int l = 0; l < (int)slabs.size(); ++l) {
            if (slabs[l].empty()) continue;
            // wavefront levels compare 16 and 32 pairs per wavefront (32 only when
            // every slab stays on the wavefront kernel), the others 16 and 32 per workgroup
            bool wave = false;
            for (const DChunks &c : slabs[l]) wave = wave || c.ch_matw != nullptr;
            const GemvList &G = lists[l];
            std::vector<DChunks> alt;
            bool alt_ok = true;
            for (const M2LChunks &C : build_chunk_slabs(G, 2 * M2LC_CH, slab_entries(G, P.opt.slab_mb))) {
                alt.push_back(upload_chunks(D, C));
                if (wave) {
                    attach_wave(D, P, C, alt.back(), nullptr);
                    alt_ok = alt_ok && alt.back().ch_matw != nullptr;
                }
            }
            size_t need = 0;
            for (const DChunks &c : alt) need = std::max(need, mfma_shm(c));
            double t16 = time(kind, slabs[l]), t32 = 1e30;
            if (wave ? alt_ok : need <= (size_t)maxsh) {
                if (!wave) set_mfma_lds(D, need);
                t32 = time(kind, alt);
            }
            const bool take = t32 < t16;
            if (take) std::swap(slabs[l], alt);
            for (DChunks &c : alt) free_chunks(D, c);
            D.autotune.push_back(
                {(double)l, (double)(take ? 2 * M2LC_CH : M2LC_CH), t16, t32, (double)kind, wave ? 1.0 : 0.0});
            if (P.opt.verbose) {
                std::fprintf(stderr, "[fdbem] autotune %s level %d (%s): 16 pairs %.3f ms, 32 pairs %.3f ms\n",
                             names[kind], l, wave ? "wavefront" : "workgroup", t16, t32);
                std::fflush(stderr);
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

void device_upload(Plan &P)
{
    Device *Dp = new Device();
    P.dev = Dp;
    Device &D = *Dp;
    HIP_CHECK(hipGetDevice(&D.device));
    D.static_part = static_scratch_address(D.device);
    D.x = dupload(D, P.px);
    D.y = dupload(D, P.py);
    D.z = dupload(D, P.pz);
    D.nx = dupload(D, P.pnx);
    D.ny = dupload(D, P.pny);
    D.nz = dupload(D, P.pnz);
    D.w = dupload(D, P.pw);
    D.perm = dupload(D, P.perm);
    {
        std::vector<PN> pnh(P.N);
        for (int64_t i = 0; i < P.N; ++i)
            pnh[i] = PN{P.px[i], P.py[i], P.pz[i], P.pnx[i], P.pny[i], P.pnz[i], 0.0, 0.0};
        D.pn = (void *)dupload(D, pnh);
    }
    D.n_leaf = (int)P.leaves.size();
    if (P.N >= (int64_t)INT32_MAX) throw std::runtime_error("more points than the near-field kernel indexes (2^31 - 1)");
    {
        // target leaves: the heaviest 2% by P2P work first, in decreasing order
        // (one wavefront each: per block of up to 64 targets, the steps of 64/nt
        // slices over the concatenated sources), so the longest wavefronts do
        // not end up in the tail; the rest in tree order, where neighbouring
        // leaves share sources in L2
        const int nl = (int)P.p2p_tgt_start.size();
        std::vector<double> work(nl, 0.0);
        for (int t = 0; t < nl; ++t) {
            const int64_t nt_all = P.p2p_tgt_end[t] - P.p2p_tgt_start[t];
            int64_t tot = 0;
            for (int e = P.p2p_ptr[t]; e < P.p2p_ptr[t + 1]; ++e) tot += P.p2p_src_end[e] - P.p2p_src_start[e];
            for (int64_t ib = 0; ib < nt_all; ib += 64) {
                const int64_t S = 64 / std::min<int64_t>(64, nt_all - ib);
                work[t] += 2.0 + (double)((tot + S - 1) / S);
            }
        }
        std::vector<int> order(nl);
        for (int t = 0; t < nl; ++t) order[t] = t;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
        {
            const int heavy = nl / 50;
            std::vector<char> first(nl, 0);
            for (int q = 0; q < heavy; ++q) first[order[q]] = 1;
            int q = heavy;
            for (int t = 0; t < nl; ++t)
                if (!first[t]) order[q++] = t;
        }
        std::vector<int64_t> ts(nl), te(nl), ss, se;
        std::vector<int> ptr(nl + 1, 0);
        ss.reserve(P.p2p_src_start.size());
        se.reserve(P.p2p_src_end.size());
        for (int q = 0; q < nl; ++q) {
            const int t = order[q];
            ts[q] = P.p2p_tgt_start[t];
            te[q] = P.p2p_tgt_end[t];
            for (int e = P.p2p_ptr[t]; e < P.p2p_ptr[t + 1]; ++e) {
                ss.push_back(P.p2p_src_start[e]);
                se.push_back(P.p2p_src_end[e]);
            }
            ptr[q + 1] = (int)ss.size();
        }
        D.p2p_ts = dupload(D, ts);
        D.p2p_te = dupload(D, te);
        D.p2p_ptr = dupload(D, ptr);
        D.p2p_ss = dupload(D, ss);
        D.p2p_se = dupload(D, se);
    }
    // templates
    const int nlev = (int)P.levels.size();
    D.n_lev = nlev;
    if (P.opt.far_field) {
        std::vector<int> ts(nlev, 0), tny(nlev, 0);
        std::vector<int64_t> yoff(nlev, 0), woff(nlev, 0);
        std::vector<double> Yall;
        std::vector<double2> Wall, Wtall;
        for (int l = 0; l < nlev; ++l) {
            const LevelTemplate &T = P.tmpl[l];
            ts[l] = T.s;
            tny[l] = (int)T.Y.size() / 3;
            yoff[l] = (int64_t)Yall.size();
            woff[l] = (int64_t)Wall.size();
            Yall.insert(Yall.end(), T.Y.begin(), T.Y.end());
            for (const cplx &v : T.W.a) Wall.push_back(make_double2(v.real(), v.imag()));
            const int ny = (int)T.Y.size() / 3;
            Wtall.insert(Wtall.end(), Wall.begin() + woff[l], Wall.end());
            if ((int64_t)T.W.a.size() == (int64_t)T.s * ny)
                for (int a = 0; a < ny; ++a)
                    for (int r = 0; r < T.s; ++r)
                        Wtall[woff[l] + a + (int64_t)r * ny] = Wall[woff[l] + r + (int64_t)a * T.s];
        }
        D.t_s = dupload(D, ts);
        D.t_ny = dupload(D, tny);
        D.t_yoff = dupload(D, yoff);
        D.t_woff = dupload(D, woff);
        D.t_Y = dupload(D, Yall);
        D.t_W = dupload(D, Wall);
        D.t_Wt = dupload(D, Wtall);
        std::vector<double2> mp(P.matpool.size());
        for (size_t i = 0; i < mp.size(); ++i) mp[i] = make_double2(P.matpool[i].real(), P.matpool[i].imag());
        D.mat = dupload(D, mp);
        int maxsh = 65536;
        (void)hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, D.device);
        // M2L mode: 3 operator chunks with per-pair results summed per output
        // (default, deterministic), 0 operator chunks with atomic adds, 1
        // per-target GEMV, 2 workgroup target tiles
        D.m2l_mode = P.opt.m2l_tile < 0 ? 1 : P.opt.m2l_tile > 1 ? 2 : P.opt.m2l_tile == 1 ? 0 : 3;
        // per-output GEMV lists: the translations of the GEMV and tile schedules
        D.m2m.resize(nlev);
        D.m2l.resize(nlev);
        D.l2l.resize(nlev);
        if (D.m2l_mode == 1 || D.m2l_mode == 2)
            for (int l = 0; l < nlev; ++l) {
                D.m2m[l] = upload_gemv(D, P.m2m_lists[l]);
                D.m2l[l] = upload_gemv(D, P.m2l_lists[l]);
                D.l2l[l] = upload_gemv(D, P.l2l_lists[l]);
            }
        if (D.m2l_mode == 3) {
            // slabs keep the scratch of per-pair results near 1 GiB
            D.m2ls.resize(nlev);
            D.m2ms.resize(nlev);
            D.l2ls.resize(nlev);
            size_t part = 0, big = 0;
            std::vector<double2> wpool;
            auto slabs = [&](const GemvList &G, std::vector<DChunks> &dst) {
                if (G.out_off.empty()) return;
                // the kernel is chosen per list, so that results do not depend on the slab size
                const bool wave = P.opt.chunk_kernel == 0 && wave_fits(G);
                for (const M2LChunks &C : build_chunk_slabs(G, M2LC_CH, slab_entries(G, P.opt.slab_mb))) {
                    dst.push_back(upload_chunks(D, C));
                    part = std::max(part, sizeof(double2) * (size_t)C.pr_pos.size() * (size_t)C.s);
                    big = std::max(big, dst.back().shm / 2);  // FP32 VALU kernel (FP64 runs on MFMA)
                    if (wave) attach_wave(D, P, C, dst.back(), &wpool);
                }
            };
            for (int l = 0; l < nlev; ++l) {
                slabs(P.m2l_lists[l], D.m2ls[l]);
                slabs(P.m2m_lists[l], D.m2ms[l]);
                slabs(P.l2l_lists[l], D.l2ls[l]);
                int64_t nch = 0, np = 0;
                for (const DChunks &c : D.m2ls[l]) nch += c.n, np += c.n_entries;
                D.tile_stats.push_back({(int64_t)D.m2ls[l].size(), nch, np, 0});
            }
            (void)big;
            if (!wpool.empty()) {
                // zero padding: masked operator loads read at most two entries past an operator's start
                wpool.resize(wpool.size() + 16, make_double2(0, 0));
                D.matw = dupload(D, wpool);
                if (P.opt.precision >= 1) {
                    std::vector<float2> wf(wpool.size());
                    for (size_t i = 0; i < wf.size(); ++i) wf[i] = make_float2((float)wpool[i].x, (float)wpool[i].y);
                    D.matwf = dupload(D, wf);
                }
                for (auto *v : {&D.m2ls, &D.m2ms, &D.l2ls})
                    for (auto &lv : *v)
                        for (DChunks &c : lv)
                            if (c.ch_matw) {
                                c.matw = D.matw;
                                c.matwf = D.matwf;
                            }
            }
            size_t mf = 0;
            for (auto *v : {&D.m2ls, &D.m2ms, &D.l2ls})
                for (const auto &lv : *v)
                    for (const DChunks &c : lv)
                        if (!c.ch_matw) mf = std::max(mf, mfma_shm(c));  // the wavefront kernel uses no LDS
            if (mf > (size_t)maxsh) throw std::runtime_error("translation operator too large for LDS");
            set_mfma_lds(D, mf);
            D.part_bytes = part;
            D.part_pipe = P.opt.serial_slabs == 0;
            if (part) D.part = dalloc<double2>(D, (D.part_pipe ? 2 : 1) * part / sizeof(double2));
        }
        if (D.m2l_mode == 0) {
            build_m2l_chunks(P, M2LC_CH);
            D.m2lc.resize(nlev);
            for (int l = 0; l < nlev; ++l) {
                D.m2lc[l] = upload_chunks(D, P.m2l_chunks[l]);
                D.tile_stats.push_back({0, (int64_t)P.m2l_chunks[l].ch_mat.size(),
                                        (int64_t)P.m2l_chunks[l].pr_tgt.size(), 0});
                if (D.m2lc[l].shm > (size_t)maxsh) D.m2l_mode = 1;
                if (D.m2lc[l].shm > 65536)
                    HIP_CHECK(hipFuncSetAttribute((const void *)k_chunks<TAG_M2L, false, double, false>,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)D.m2lc[l].shm));
            }
            P.m2l_chunks.clear();
            // up and down passes by operator chunks as well
            D.m2mc.resize(nlev);
            D.l2lc.resize(nlev);
            for (int l = 0; l < nlev; ++l) {
                D.m2mc[l] = upload_chunks(D, build_chunks(P.m2m_lists[l], M2LC_CH));
                D.l2lc[l] = upload_chunks(D, build_chunks(P.l2l_lists[l], M2LC_CH));
                for (const DChunks *c : {&D.m2mc[l], &D.l2lc[l]})
                    if (c->shm > (size_t)maxsh) throw std::runtime_error("translation operator too large for LDS");
            }
        }
        if (D.m2l_mode == 2) {
            // deterministic tiles: the largest tile whose LDS footprint fits one workgroup
            int tile = P.opt.m2l_tile, chunk = std::min(32, tile);
            auto fits = [&](int t, int c) {
                for (int l = 0; l < nlev; ++l) {
                    const GemvList &G = P.m2l_lists[l];
                    if (G.out_off.empty()) continue;
                    int rmax = 1;
                    for (int r : G.rank) rmax = std::max(rmax, r);
                    if (sizeof(double2) * ((size_t)(t + c) * G.rows + (size_t)c * rmax) > (size_t)maxsh) return false;
                }
                return true;
            };
            while (tile > 4 && !fits(tile, chunk)) {
                tile /= 2;
                chunk = std::min(chunk, tile);
            }
            if (!fits(tile, chunk)) D.m2l_mode = 1;
        }
        if (D.m2l_mode == 2) {
            int tile = P.opt.m2l_tile, chunk = std::min(32, tile);
            auto fits = [&](int t, int c) {
                for (int l = 0; l < nlev; ++l) {
                    const GemvList &G = P.m2l_lists[l];
                    if (G.out_off.empty()) continue;
                    int rmax = 1;
                    for (int r : G.rank) rmax = std::max(rmax, r);
                    if (sizeof(double2) * ((size_t)(t + c) * G.rows + (size_t)c * rmax) > (size_t)maxsh) return false;
                }
                return true;
            };
            while (tile > 4 && !fits(tile, chunk)) {
                tile /= 2;
                chunk = std::min(chunk, tile);
            }
            build_m2l_tiles(P, tile, chunk);
            D.m2lt.resize(nlev);
            int cus = 256;
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, D.device);
            size_t part = 0;
            for (int l = 0; l < nlev; ++l) {
                D.m2lt[l] = upload_tiles(D, P.m2l_tiles[l]);
                DTiles &T = D.m2lt[l];
                D.tile_stats.push_back({(int64_t)P.m2l_tiles[l].tile_ntgt.size(), (int64_t)P.m2l_tiles[l].ch_mat.size(),
                                        (int64_t)P.m2l_tiles[l].pr_tl.size(), 0});
                if (T.n_tiles) {
                    // enough workgroups to fill the chip: split tiles into segments
                    T.nseg = std::max(1, std::min(16, (8 * cus + T.n_tiles - 1) / T.n_tiles));
                    if (T.nseg > 1) part = std::max(part, (size_t)T.n_tiles * T.nseg * T.tile * T.s);
                }
                D.tile_stats.back()[3] = T.nseg;
                if (D.m2lt[l].shm > 65536)
                    HIP_CHECK(hipFuncSetAttribute((const void *)k_m2l_tile,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)D.m2lt[l].shm));
            }
            P.m2l_tiles.clear();
            if (part) D.m2l_part = dalloc<double2>(D, part);
        }
        D.s2m = upload_leaf(D, P, P.s2m_tasks);
        D.l2t = upload_leaf(D, P, P.l2t_tasks);
        if (D.s2m.n && s2m_shm<double>(P) > 65536) {
            if (s2m_shm<double>(P) > (size_t)maxsh) throw std::runtime_error("S2M templates too large for LDS");
            HIP_CHECK(hipFuncSetAttribute((const void *)k_s2m<double, OpC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)s2m_shm<double>(P)));
            HIP_CHECK(hipFuncSetAttribute((const void *)k_s2m<float, OpCf>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)s2m_shm<float>(P)));
        }
        if (D.l2t.n) {
            const size_t lsh = l2t_shm<double>(P);
            if (lsh > (size_t)maxsh) throw std::runtime_error("L2T templates too large for LDS");
            if (lsh > 65536) {
                HIP_CHECK(hipFuncSetAttribute((const void *)k_l2t<double, OpC>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lsh));
                HIP_CHECK(hipFuncSetAttribute((const void *)k_l2t<float, OpCf>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)l2t_shm<float>(P)));
            }
        }
        D.n_od = P.out_total;
        D.n_id = P.in_total;
        D.prec = P.opt.precision;
        if (D.prec >= 1) {
            if (D.m2l_mode != 0 && D.m2l_mode != 3)
                throw std::runtime_error("FP32 far field needs the operator-chunk or output-tile schedule");
            std::vector<float2> mf(P.matpool.size()), wf;
            for (size_t i = 0; i < mf.size(); ++i)
                mf[i] = make_float2((float)P.matpool[i].real(), (float)P.matpool[i].imag());
            D.matf = dupload(D, mf);
            for (int l = 0; l < nlev; ++l)
                for (const cplx &v : P.tmpl[l].W.a) wf.push_back(make_float2((float)v.real(), (float)v.imag()));
            D.t_Wf = dupload(D, wf);
            std::vector<float2> wtf(wf.size());
            for (int l = 0, off = 0; l < nlev; ++l) {
                const LevelTemplate &T = P.tmpl[l];
                const int ny = (int)T.Y.size() / 3;
                const bool full = (int64_t)T.W.a.size() == (int64_t)T.s * ny;
                for (size_t e = 0; e < T.W.a.size(); ++e) {
                    const size_t r = full ? e % T.s : 0, a = full ? e / T.s : e;
                    const cplx v = T.W.a[e];
                    wtf[off + (full ? a + r * ny : e)] = make_float2((float)v.real(), (float)v.imag());
                }
                off += (int)T.W.a.size();
            }
            D.t_Wtf = dupload(D, wtf);
            D.odf = dalloc<float2>(D, D.n_od);
            D.idf = dalloc<float2>(D, D.n_id);
        }
        if (D.prec != 1) {
            D.od = dalloc<double2>(D, D.n_od);
            D.id = dalloc<double2>(D, D.n_id);
        }
    }
    D.dens = dalloc<double2>(D, P.N);
    D.res = dalloc<double2>(D, P.N);
    if (P.n_elem > 0 && (P.opt.corrections & 3)) {
        const auto t0 = std::chrono::steady_clock::now();
        build_corrections_device(P, D);
        P.t_setup_corr = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (P.opt.verbose) {
            std::fprintf(stderr, "[fdbem] near-field corrections %.2f s (%lld element blocks)\n", P.t_setup_corr,
                         (long long)P.corr_blocks);
            std::fflush(stderr);
        }
    }
    D.ev.assign((size_t)Device::kRing * 10, nullptr);
    for (auto &e : D.ev) HIP_CHECK(hipEventCreate(&e));
    if (P.opt.autotune && P.opt.far_field && D.m2l_mode == 3) autotune_m2l(P, D);
}

void device_free(Plan &P)
{
    if (!P.dev) return;
    Device &D = *P.dev;
    graph_release(D);
    for (void *p : D.allocs) (void)hipFree(p);
    for (void *p : {(void *)D.gm_V, (void *)D.gm_w, (void *)D.gm_r, (void *)D.gm_h, (void *)D.gm_red_c,
                    (void *)D.gm_z, (void *)D.gm_t})
        if (p) (void)hipFree(p);
    for (auto &e : D.ev)
        if (e) (void)hipEventDestroy(e);
    delete P.dev;
    P.dev = nullptr;
}

// coefficients of K = (c0 + c1 d/dn_y)(d0 + d1 d/dn_x) G with alpha = i / ka
static OpC op_coef(int op, double ka)
{
    const double2 z = make_double2(0, 0), one = make_double2(1, 0), al = make_double2(0, 1.0 / ka);
    OpC c;
    switch (op) {
    case 0:  // RAW_H
    case 3:  // BM_H
        c.c0 = z; c.c1 = one; c.d0 = one; c.d1 = al; break;
    case 1:  // RAW_G
    case 4:  // BM_G
        c.c0 = one; c.c1 = z; c.d0 = one; c.d1 = al; break;
    default:  // RAW_T1
        c.c0 = one; c.c1 = al; c.d0 = one; c.d1 = z; break;
    }
    auto mul = [](double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); };
    c.cd00 = mul(c.c0, c.d0);
    c.cd10 = mul(c.c1, c.d0);
    c.cd01 = mul(c.c0, c.d1);
    c.cd11 = mul(c.c1, c.d1);
    return c;
}


template <int TAG>
static void run_gemv(const DGemv &g, const double2 *mat, const double2 *in, double2 *out, hipStream_t st)
{
    if (g.n_out == 0) return;
    const size_t shm = sizeof(double2) * (g.cols + std::max(g.max_rank, 1));
    hipLaunchKernelGGL(k_gemv<TAG>, dim3(g.n_out), dim3(GEMV_BLOCK), shm, st, g.out_off, g.ptr, g.in_off, g.mat_off, g.rank,
                       g.rows, g.cols, g.trans, mat, in, out);
}

template <typename R, typename O>
static void launch_p2p(Plan &P, Device &D, int op, hipStream_t st)
{
    const int opk = (op == 0 || op == 3) ? OPK_H : (op == 1 || op == 4) ? OPK_G : OPK_T1;
    // one 64-lane workgroup per target leaf: a finished wavefront frees its
    // slot at once instead of waiting for the slowest leaf of its group
    const dim3 g(D.n_leaf), b(64);
    const double ai = 1.0 / P.opt.alpha_k(P.k);
    if (opk == OPK_H)
        hipLaunchKernelGGL((k_p2p<OPK_H, R>), g, b, 0, st, D.n_leaf, D.p2p_ts, D.p2p_te, D.p2p_ptr, D.p2p_ss, D.p2p_se,
                           (const PN *)D.pn, D.res, P.k, ai);
    else if (opk == OPK_G)
        hipLaunchKernelGGL((k_p2p<OPK_G, R>), g, b, 0, st, D.n_leaf, D.p2p_ts, D.p2p_te, D.p2p_ptr, D.p2p_ss, D.p2p_se,
                           (const PN *)D.pn, D.res, P.k, ai);
    else
        hipLaunchKernelGGL((k_p2p<OPK_T1, R>), g, b, 0, st, D.n_leaf, D.p2p_ts, D.p2p_te, D.p2p_ptr, D.p2p_ss,
                           D.p2p_se, (const PN *)D.pn, D.res, P.k, ai);
}

template <int TAG, bool TRANS, typename R>
static void launch_chunks(const DChunks &C, int cols, const typename Cx<R>::T *mat, const typename Cx<R>::T *in,
                          typename Cx<R>::T *out, hipStream_t st)
{
    if (!C.n) return;
    const size_t shm = C.shm * sizeof(typename Cx<R>::T) / sizeof(double2);
    hipLaunchKernelGGL((k_chunks<TAG, TRANS, R, false>), dim3((C.n + M2LC_WAVES - 1) / M2LC_WAVES),
                       dim3(64 * M2LC_WAVES), shm, st, C.n, C.s, cols, C.rmax, C.ch_mat, C.ch_rank, C.ch_pptr, C.pr_tgt,
                       C.pr_src, mat, in, out, (const int64_t *)nullptr, (typename Cx<R>::T *)nullptr);
}

// row-major operator pool of a slab on the wavefront kernel (null: workgroup kernel)
template <typename R>
static const typename Cx<R>::T *wave_pool(const DChunks &c);
template <>
const double2 *wave_pool<double>(const DChunks &c)
{
    return c.ch_matw ? c.matw : nullptr;
}
template <>
const float2 *wave_pool<float>(const DChunks &c)
{
    return c.ch_matw ? c.matwf : nullptr;
}

// workgroups of the wavefront kernel for n chunks: four chunks each, a multiple of the XCD count
static int wave_grid(int n)
{
    const int nb = (n + 3) / 4;
    return ((nb + kXcds - 1) / kXcds) * kXcds;
}

// partial-sum schedule: per slab, per-pair results into the scratch, then the per-output sums
template <int TAG, bool TRANS, typename R>
static void launch_slabs(const std::vector<DChunks> &S, void *part, const typename Cx<R>::T *mat,
                         const typename Cx<R>::T *in, typename Cx<R>::T *out, hipStream_t st)
{
    using C = typename Cx<R>::T;
    for (const DChunks &c : S) {
        if (!c.n) continue;
        const size_t shm = mfma_shm(c) * sizeof(R) / sizeof(double);
        const unsigned grid = (unsigned)(((c.n + kXcds - 1) / kXcds) * kXcds);
        if (const C *mw = wave_pool<R>(c))
            launch_wave<R, TAG>(c, dim3(wave_grid(c.n)), st, 0, 0, 0, nullptr, nullptr, nullptr, nullptr, mw, in,
                                (C *)part);
        else if (c.pw == 32)
            hipLaunchKernelGGL((k_chunks_mfma<R, TRANS, 2, TAG>), dim3(grid), dim3(64 * M2LC_WAVES), shm, st, c.n, c.s,
                               c.cols, c.rmax, c.ch_mat, c.ch_rank, c.ch_pptr, c.pr_src, c.pr_pos, mat, in, (C *)part);
        else
            hipLaunchKernelGGL((k_chunks_mfma<R, TRANS, 1, TAG>), dim3(grid), dim3(64 * M2LC_WAVES), shm, st, c.n, c.s,
                               c.cols, c.rmax, c.ch_mat, c.ch_rank, c.ch_pptr, c.pr_src, c.pr_pos, mat, in, (C *)part);
        hipLaunchKernelGGL((k_seg_sum<R, TAG>), dim3((c.n_out + 3) / 4), dim3(256), 0, st, c.n_out, c.s, c.red_out,
                           c.red_ptr, (const C *)part, out);
    }
}

// Slabs in a pipeline over two scratch buffers: launch j runs the chunks of
// slab j and the sums of slab j - 1 (k_chunks_seg); the sums of the last slab
// stay pending in `pend` so that a caller can overlap them with the next
// list's chunks when that list does not read their outputs (M2L levels), or
// flush them (M2M and L2L levels).
template <typename R>
struct PendingSum {
    const DChunks *c = nullptr;
    void *part = nullptr;
    typename Cx<R>::T *out = nullptr;
};

template <typename R, int TAG>
static void flush_sum(PendingSum<R> &pend, hipStream_t st)
{
    using C = typename Cx<R>::T;
    if (!pend.c) return;
    const DChunks &c = *pend.c;
    hipLaunchKernelGGL((k_seg_sum<R, TAG>), dim3((c.n_out + 3) / 4), dim3(256), 0, st, c.n_out, c.s, c.red_out,
                       c.red_ptr, (const C *)pend.part, pend.out);
    pend = PendingSum<R>();
}

template <int TAG, bool TRANS, typename R>
static void launch_slabs_pipe(const std::vector<DChunks> &S, void *const part2[2], int &turn, PendingSum<R> &pend,
                              const typename Cx<R>::T *mat, const typename Cx<R>::T *in, typename Cx<R>::T *out,
                              hipStream_t st)
{
    using C = typename Cx<R>::T;
    for (const DChunks &c : S) {
        if (!c.n) continue;
        void *part = part2[turn];
        const size_t shm = mfma_shm(c) * sizeof(R) / sizeof(double);
        const int chunk_grid = (int)(((c.n + kXcds - 1) / kXcds) * kXcds);
        int n_seg = 0, n_out_prev = 0, s_prev = 0;
        const int64_t *ro = nullptr, *rp = nullptr;
        const C *prev = nullptr;
        C *out_prev = nullptr;
        if (pend.c) {
            n_out_prev = pend.c->n_out;
            s_prev = pend.c->s;
            ro = pend.c->red_out;
            rp = pend.c->red_ptr;
            prev = (const C *)pend.part;
            out_prev = pend.out;
            n_seg = (int)((((n_out_prev + 3) / 4) + kXcds - 1) / kXcds * kXcds);
        }
        const dim3 grid((unsigned)(n_seg + chunk_grid)), block(64 * M2LC_WAVES);
        if (const C *mw = wave_pool<R>(c))
            launch_wave<R, TAG>(c, dim3((unsigned)(n_seg + wave_grid(c.n))), st, n_seg, n_out_prev, s_prev, ro, rp,
                                prev, out_prev, mw, in, (C *)part);
        else if (c.pw == 32)
            hipLaunchKernelGGL((k_chunks_seg<R, TRANS, 2, TAG>), grid, block, shm, st, n_seg, n_out_prev, s_prev, ro, rp,
                               prev, out_prev, c.n, c.s, c.cols, c.rmax, c.ch_mat, c.ch_rank, c.ch_pptr, c.pr_src,
                               c.pr_pos, mat, in, (C *)part);
        else
            hipLaunchKernelGGL((k_chunks_seg<R, TRANS, 1, TAG>), grid, block, shm, st, n_seg, n_out_prev, s_prev, ro, rp,
                               prev, out_prev, c.n, c.s, c.cols, c.rmax, c.ch_mat, c.ch_rank, c.ch_pptr, c.pr_src,
                               c.pr_pos, mat, in, (C *)part);
        pend.c = &c;
        pend.part = part;
        pend.out = out;
        turn ^= 1;
    }
}

template <typename R, typename O>
static void launch_s2m(Plan &P, Device &D, const O &c, const typename Cx<R>::T *tW, typename Cx<R>::T *od,
                       hipStream_t st)
{
    if (!D.s2m.n) return;
    hipLaunchKernelGGL((k_s2m<R, O>), dim3(D.s2m.n_groups), dim3(LEAF_BLOCK), s2m_shm<R>(P), st, D.s2m.gptr,
                       D.s2m.start, D.s2m.end, D.s2m.slot, D.s2m.tmpl, D.s2m.center, D.t_s, D.t_ny, D.t_yoff,
                       D.t_woff, D.t_Y, tW, D.x, D.y, D.z, D.nx, D.ny, D.nz, D.dens, od, P.k, c,
                       std::max(P.max_Y_leaf, 1));
}

template <typename R, typename O>
static void launch_l2t(Plan &P, Device &D, const O &c, const typename Cx<R>::T *tWt, const typename Cx<R>::T *id,
                       hipStream_t st)
{
    if (!D.l2t.n) return;
    hipLaunchKernelGGL((k_l2t<R, O>), dim3(D.l2t.n_groups), dim3(LEAF_BLOCK), l2t_shm<R>(P), st, D.l2t.gptr,
                       D.l2t.start, D.l2t.end, D.l2t.slot, D.l2t.tmpl, D.l2t.center, D.t_s, D.t_ny, D.t_yoff,
                       D.t_woff, D.t_Y, tWt, D.x, D.y, D.z, D.nx, D.ny, D.nz, id, D.res, P.k, c,
                       std::max(P.max_Y_leaf, 1), std::max(P.max_s, 1));
}

// S2M .. L2T in working precision R (operator-chunk schedule)
template <typename R, typename O>
static void far_field_chunks(Plan &P, Device &D, const O &c, const typename Cx<R>::T *mat, const typename Cx<R>::T *tW,
                             const typename Cx<R>::T *tWt, typename Cx<R>::T *od, typename Cx<R>::T *id,
                             void *part, void *const *part2, hipEvent_t *ev, hipStream_t st)
{
    using C = typename Cx<R>::T;
    if (D.n_od) hipLaunchKernelGGL(k_fill_zero<C>, dim3(nblk(D.n_od, 256)), dim3(256), 0, st, od, D.n_od);
    if (D.n_id) hipLaunchKernelGGL(k_fill_zero<C>, dim3(nblk(D.n_id, 256)), dim3(256), 0, st, id, D.n_id);
    launch_s2m<R, O>(P, D, c, tW, od, st);
    if (ev) HIP_CHECK(hipEventRecord(ev[3], st));
    const bool slabs = D.m2l_mode == 3;
    // two scratch buffers: pipelined slabs (the second buffer follows the first)
    const bool pipe = slabs && part2 != nullptr;
    int turn = 0;
    PendingSum<R> pend;
    for (int l = D.n_lev - 2; l >= 0; --l) {
        if (pipe) {
            launch_slabs_pipe<TAG_M2M, false, R>(D.m2ms[l], part2, turn, pend, mat, od, od, st);
            flush_sum<R, TAG_M2M>(pend, st);  // the next level's M2M reads these outputs
        } else if (slabs)
            launch_slabs<TAG_M2M, false, R>(D.m2ms[l], part, mat, od, od, st);
        else
            launch_chunks<TAG_M2M, false, R>(D.m2mc[l], D.m2mc[l].cols, mat, od, od, st);
    }
    if (ev) HIP_CHECK(hipEventRecord(ev[4], st));
    for (int l = 0; l < D.n_lev; ++l) {
        if (pipe)
            launch_slabs_pipe<TAG_M2L, false, R>(D.m2ls[l], part2, turn, pend, mat, od, id, st);  // levels independent
        else if (slabs)
            launch_slabs<TAG_M2L, false, R>(D.m2ls[l], part, mat, od, id, st);
        else
            launch_chunks<TAG_M2L, false, R>(D.m2lc[l], D.m2lc[l].s, mat, od, id, st);
    }
    if (pipe) flush_sum<R, TAG_M2L>(pend, st);
    if (ev) HIP_CHECK(hipEventRecord(ev[5], st));
    for (int l = 1; l < D.n_lev; ++l) {
        if (pipe) {
            launch_slabs_pipe<TAG_L2L, true, R>(D.l2ls[l], part2, turn, pend, mat, id, id, st);
            flush_sum<R, TAG_L2L>(pend, st);  // the next level's L2L reads these outputs
        } else if (slabs)
            launch_slabs<TAG_L2L, true, R>(D.l2ls[l], part, mat, id, id, st);
        else
            launch_chunks<TAG_L2L, true, R>(D.l2lc[l], D.l2lc[l].cols, mat, id, id, st);
    }
    if (ev) HIP_CHECK(hipEventRecord(ev[6], st));
    launch_l2t<R, O>(P, D, c, tWt, id, st);
}

void device_matvec(Plan &P, int op, const double2 *in, double2 *out, hipStream_t st, void *part)
{
    Device &D = *P.dev;
    // the plan's scratch holds two slab buffers (pipelined slabs); a caller's
    // buffer holds one unless it is twice the slab size
    void *part2[2] = {nullptr, nullptr};
    void *const *pp2 = nullptr;
    if (!part) {
        part = D.part;
        if (D.part_pipe) {
            part2[0] = D.part;
            part2[1] = (char *)D.part + D.part_bytes;
            pp2 = part2;
        }
    }
    const int64_t N = P.N;
    // low byte: operator; FDA_OP_FP32 (0x100) selects the FP32 far field and
    // near field on plans built with both precisions
    const bool f32 = D.prec == 1 || (D.prec == 2 && (op & 0x100));
    op &= 0xff;
    const OpC c = op_coef(op, P.opt.alpha_k(P.k));
    const bool tm = D.timing != 0;
    hipEvent_t *ev = tm ? &D.ev[(size_t)(D.ring_pos % Device::kRing) * 10] : nullptr;
    if (tm) HIP_CHECK(hipEventRecord(ev[0], st));
    hipLaunchKernelGGL(k_permute_in, dim3(nblk(N, 256)), dim3(256), 0, st, in, D.perm, D.w, D.dens, (double *)D.pn, N);
    if (tm) HIP_CHECK(hipEventRecord(ev[1], st));
    if (f32)
        launch_p2p<float, OpCf>(P, D, op, st);
    else
        launch_p2p<double, OpC>(P, D, op, st);
    if (tm) HIP_CHECK(hipEventRecord(ev[2], st));
    if (P.opt.far_field && f32) {
        const OpCf cf = {make_float2((float)c.c0.x, (float)c.c0.y), make_float2((float)c.c1.x, (float)c.c1.y),
                         make_float2((float)c.d0.x, (float)c.d0.y), make_float2((float)c.d1.x, (float)c.d1.y)};
        far_field_chunks<float, OpCf>(P, D, cf, D.matf, D.t_Wf, D.t_Wtf, D.odf, D.idf, part, pp2, ev, st);
    } else if (P.opt.far_field && (D.m2l_mode == 0 || D.m2l_mode == 3)) {
        far_field_chunks<double, OpC>(P, D, c, D.mat, D.t_W, D.t_Wt, D.od, D.id, part, pp2, ev, st);
    } else if (P.opt.far_field) {
        if (D.n_od) hipLaunchKernelGGL(k_fill_zero<double2>, dim3(nblk(D.n_od, 256)), dim3(256), 0, st, D.od, D.n_od);
        if (D.n_id) hipLaunchKernelGGL(k_fill_zero<double2>, dim3(nblk(D.n_id, 256)), dim3(256), 0, st, D.id, D.n_id);
        launch_s2m<double, OpC>(P, D, c, D.t_W, D.od, st);
        if (tm) HIP_CHECK(hipEventRecord(ev[3], st));
        for (int l = D.n_lev - 2; l >= 0; --l) run_gemv<TAG_M2M>(D.m2m[l], D.mat, D.od, D.od, st);
        if (tm) HIP_CHECK(hipEventRecord(ev[4], st));
        for (int l = 0; l < D.n_lev; ++l) {
            if (D.m2l_mode == 2) {
                const DTiles &T = D.m2lt[l];
                if (T.n_tiles) {
                    hipLaunchKernelGGL(k_m2l_tile, dim3(T.n_tiles * T.nseg), dim3(M2L_BLOCK), T.shm, st, T.s, T.rmax,
                                       T.tile, T.chunk, T.nseg, D.m2l_part, T.tgt_off, T.tile_ntgt, T.tile_cptr,
                                       T.ch_mat, T.ch_rank, T.ch_pptr, T.pr_tl, T.pr_src, D.mat, D.od, D.id);
                    if (T.nseg > 1)
                        hipLaunchKernelGGL(k_m2l_reduce, dim3(T.n_tiles), dim3(256), 0, st, T.s, T.tile, T.nseg,
                                           D.m2l_part, T.tgt_off, T.tile_ntgt, D.id);
                }
            } else
                run_gemv<TAG_M2L>(D.m2l[l], D.mat, D.od, D.id, st);
        }
        if (tm) HIP_CHECK(hipEventRecord(ev[5], st));
        for (int l = 1; l < D.n_lev; ++l) run_gemv<TAG_L2L>(D.l2l[l], D.mat, D.id, D.id, st);
        if (tm) HIP_CHECK(hipEventRecord(ev[6], st));
        launch_l2t<double, OpC>(P, D, c, D.t_Wt, D.id, st);
    } else if (tm) {
        for (int e = 3; e <= 6; ++e) HIP_CHECK(hipEventRecord(ev[e], st));
    }
    if (tm) HIP_CHECK(hipEventRecord(ev[7], st));
    hipLaunchKernelGGL(k_permute_out, dim3(nblk(N, 256)), dim3(256), 0, st, D.res, D.perm, in, op == 3 ? 0.5 : 0.0, out, N);
    if (tm) HIP_CHECK(hipEventRecord(ev[8], st));
    // the near-field correction stays in FP64 in both precisions
    if (op == 3 && D.corr.val)
        hipLaunchKernelGGL(k_corr, dim3(nblk(N, 256)), dim3(256), 0, st, D.corr.rp, D.corr.blk, D.corr.val, in, out, N);
    if (op == 4 && D.corrg.val)
        hipLaunchKernelGGL(k_corr, dim3(nblk(N, 256)), dim3(256), 0, st, D.corrg.rp, D.corrg.blk, D.corrg.val, in, out,
                           N);
    if (tm) {
        HIP_CHECK(hipEventRecord(ev[9], st));
        D.ring_pos++;
        D.ring_count++;
    }
    HIP_CHECK(hipGetLastError());
}

// Average the per-phase times of the timed mat-vecs recorded since the last
// call (at most the ring size), then start a new window.
void device_phase_average(Plan &P)
{
    Device &D = *P.dev;
    const int n = std::min(D.ring_count, Device::kRing);
    for (int t = 0; t < 8; ++t) D.phase_ms[t] = 0.0;
    if (n == 0) return;
    const int a[8] = {1, 2, 3, 4, 5, 6, 8, 0}, b[8] = {2, 3, 4, 5, 6, 7, 9, 1};
    for (int q = 0; q < n; ++q) {
        const int slot = (D.ring_pos - 1 - q + Device::kRing * 4) % Device::kRing;
        hipEvent_t *ev = &D.ev[(size_t)slot * 10];
        HIP_CHECK(hipEventSynchronize(ev[9]));
        float ms;
        for (int t = 0; t < 7; ++t) {
            HIP_CHECK(hipEventElapsedTime(&ms, ev[a[t]], ev[b[t]]));
            D.phase_ms[t] += ms / n;
        }
        float m0, m1;
        HIP_CHECK(hipEventElapsedTime(&m0, ev[0], ev[1]));
        HIP_CHECK(hipEventElapsedTime(&m1, ev[7], ev[8]));
        D.phase_ms[7] += (m0 + m1) / n;
    }
    D.ring_count = 0;
}

void device_rhs_plane_wave(Plan &P, const double d[3], double2 *rhs, hipStream_t st)
{
    Device &D = *P.dev;
    hipLaunchKernelGGL(k_plane_wave, dim3(nblk(P.N, 256)), dim3(256), 0, st, D.x, D.y, D.z, D.nx, D.ny, D.nz, D.perm,
                       P.k, P.opt.coupling, d[0], d[1], d[2], rhs, P.N);
    HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------- static scratch
// Per-pair translation results of the allocation-free mat-vec live in this
// file-scope device array instead of the plan's slab buffer.  Each device the
// library runs on holds its own copy for the life of the process.  In host
// code the name is only a stand-in: the device address comes from
// hipGetSymbolAddress, looked up once per device at plan set-up.
static __device__ __align__(256) double2 scratch[kStaticScratchBytes / sizeof(double2)];

void *static_scratch_address(int device)
{
    static std::mutex mu;
    static std::map<int, void *> addr;  // device -> address of its copy
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) return it->second;
    int cur = -1;
    HIP_CHECK(hipGetDevice(&cur));
    if (cur != device) throw std::runtime_error("static scratch looked up with another device current");
    void *p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw std::runtime_error("no device address for the static scratch");
    addr[device] = p;
    return p;
}

// The mat-vec of device_matvec with the per-pair results in the static
// scratch.  Everything it reads or writes besides the vectors was allocated
// when the plan was built; the scratch rows are written before they are read,
// so nothing has to be cleared.
void device_matvec_static(Plan &P, int op, const double2 *in, double2 *out, hipStream_t st)
{
    Device &D = *P.dev;
    if (D.m2l_mode != 3 && D.m2l_mode != 0)
        throw std::invalid_argument("the allocation-free mat-vec needs the operator-chunk translation schedule");
    if (D.part_bytes > kStaticScratchBytes)
        throw std::invalid_argument("the plan's translation slabs need " + std::to_string(D.part_bytes) +
                                    " bytes of scratch, more than the static " + std::to_string(kStaticScratchBytes) +
                                    " bytes: build it with slab_mb <= " + std::to_string(kStaticScratchBytes >> 20));
    if (!D.static_part) throw std::runtime_error("static scratch address missing");
    device_matvec(P, op, in, out, st, D.static_part);
}

// Right-hand side of a Neumann (radiation) problem: (S + alpha M) q through
// the corrected G operator, minus alpha c q with c = 1/2.
void device_rhs_neumann(Plan &P, const double2 *q, double2 *rhs, hipStream_t st)
{
    device_matvec(P, 4 /* FDA_OP_BM_G */, q, rhs, st);
    // alpha = i coupling / k, so alpha / 2 = (0, coupling / (2 k))
    hipLaunchKernelGGL(k_sub_scaled, dim3(nblk(P.N, 256)), dim3(256), 0, st, q, 0.0, 0.5 * P.opt.coupling / P.k, rhs,
                       P.N);
    HIP_CHECK(hipGetLastError());
}

}  // namespace fdbem
