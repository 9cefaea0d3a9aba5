// Equivalent/check point templates, pseudo-inverses and the compressed
// translation operators of the fast directional algorithm.
//
// * Low frequency (w < lambda): kernel-independent surface grids as in the
//   kernel-independent FMM: equivalent points on a cube surface of half-width
//   1.05 w/2, check points on one of half-width 2.95 w/2 (section 3.1.2).
// * High frequency (w = m lambda): one template for direction +x, rotated to
//   each wedge; the pseudo-inverse is shared by all wedges (section 3.1.2).
//   Check points fill the cone of the wedge (cell of the face grid plus the
//   angular radius of a target cube at the smallest interaction distance)
//   between that distance and the far field; equivalent points are a skeleton
//   of the cube's ball selected by a randomised pivoted Gram-Schmidt on the
//   check-to-candidate interaction matrix.
// * R = G(check, equivalent) = U S V^H, truncated at sigma_i >= eps sigma_1
//   (eqs. eq_svdr, eq_invr).  Compressed operators (eqs. eq_cmps .. eq_cmpt):
//     S2M:  S~ = S~^-1 U~^H E_up           (applied on the fly from W = S~^-1 U~^H)
//     M2M:  M~ = W_parent E(parent check, child equivalent) V~_child
//     M2L:  K~ = V~^T G(target equivalent, source equivalent) V~
//           (incoming check points are the outgoing equivalent points, so
//            U~_dn^H = V~^T, section 3.2 transpose identities)
//     L2L:  L~ = M~^T
//     L2T:  T~ = E_dn conj(U~) S~^-1 = E_dn W^T
// * Low-rank M2L (eq. eq_lrdk): K~ ~= U^ V^ with V^ = S^ Q^^H, truncating
//   sigma < eps sigma_1; used iff its rank r < s/2, else K~ is applied.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>
#include <stdexcept>

#include "plan.hpp"

namespace fdbem {

namespace {

double svd_eps(const Plan &P) { return P.opt.svd_eps > 0 ? P.opt.svd_eps : P.eps; }
// High-frequency orbit templates fit the field on a skeleton of the points
// where it is evaluated; between those points the error is about three times
// the truncation, so by default they truncate at eps / 3.
double hf_svd_eps(const Plan &P) { return P.opt.svd_eps > 0 ? P.opt.svd_eps : P.eps / 3.0; }
double lr_eps(const Plan &P) { return P.opt.lowrank_eps > 0 ? P.opt.lowrank_eps : P.eps; }

std::vector<double> cube_surface(int p, double a)
{
    std::vector<double> pts;
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            for (int l = 0; l < p; ++l) {
                if (i != 0 && i != p - 1 && j != 0 && j != p - 1 && l != 0 && l != p - 1) continue;
                pts.push_back(-a + 2.0 * a * i / (p - 1));
                pts.push_back(-a + 2.0 * a * j / (p - 1));
                pts.push_back(-a + 2.0 * a * l / (p - 1));
            }
    return pts;
}

// quasi-uniform points on the cap {theta <= th} around +x (Fibonacci lattice)
void cap_points(int n, double th, double radius, std::vector<double> &out)
{
    const double ga = M_PI * (3.0 - std::sqrt(5.0));
    const double cmin = std::cos(th);
    for (int i = 0; i < n; ++i) {
        const double c = 1.0 - (1.0 - cmin) * (i + 0.5) / n;
        const double s = std::sqrt(std::max(0.0, 1.0 - c * c));
        const double ph = ga * i;
        out.push_back(radius * c);
        out.push_back(radius * s * std::cos(ph));
        out.push_back(radius * s * std::sin(ph));
    }
}

void finish_template(LevelTemplate &T, double k, double eps)
{
    const int ny = (int)T.Y.size() / 3, nx = (int)T.X.size() / 3;
    CMat R(ny, nx);
    for (int j = 0; j < nx; ++j)
        for (int i = 0; i < ny; ++i) R(i, j) = kernel_G(&T.Y[3 * i], &T.X[3 * j], k);
    SVD d = svd(R);
    const int s = std::max(1, truncation_rank(d.s, eps));
    T.s = s;
    T.sing = d.s;
    T.Vt = CMat(nx, s);
    T.W = CMat(s, ny);
    for (int c = 0; c < s; ++c) {
        for (int i = 0; i < nx; ++i) T.Vt(i, c) = d.V(i, c);
        for (int i = 0; i < ny; ++i) T.W(c, i) = std::conj(d.U(i, c)) / d.s[c];
    }
}

// The original method of the paper (Table 1's comparison) keeps the
// equivalent densities themselves: basis V~ -> I (|X| x |X|, zero columns
// up to s_out) and W -> V~ S~^-1 U~^H = R^+ (rows past |X| zero), so every
// translation acts in dimension |X| with the uncompressed R^+ (eq. eq_invr)
// and K; the products equal those of the reduced basis up to rounding.
void to_original_basis(CMat &Vt, CMat &W, int &s, int nx, int s_out = 0)
{
    const int so = std::max(nx, s_out);
    const int ny = W.n;
    CMat I(nx, so), Rp(so, ny);
    for (int i = 0; i < nx; ++i) I(i, i) = 1.0;
    for (int c = 0; c < s; ++c)
        for (int j = 0; j < ny; ++j) {
            const cplx wv = W(c, j);
            if (wv == cplx(0.0)) continue;
            for (int i = 0; i < nx; ++i) Rp(i, j) += Vt(i, c) * wv;
        }
    Vt = std::move(I);
    W = std::move(Rp);
    s = so;
}

LevelTemplate lf_template(const Plan &P, double w)
{
    LevelTemplate T;
    T.hf = false;
    T.w = w;
    int p = P.opt.lf_grid;
    if (p <= 0) p = std::max(4, (int)std::ceil(-std::log10(svd_eps(P))) + 4);
    T.X = cube_surface(p, 1.05 * 0.5 * w);
    T.Y = cube_surface(p, 2.95 * 0.5 * w);
    finish_template(T, P.k, svd_eps(P));
    if (P.opt.original) to_original_basis(T.Vt, T.W, T.s, (int)T.X.size() / 3);
    return T;
}

double cell_angle(int m)
{
    // largest angle between a face cell's central direction and its corners
    double worst = 0;
    for (int iu = 0; iu < m; ++iu)
        for (int it = 0; it < m; ++it) {
            const double cu = (2.0 * iu + 1.0 - m) / m, ct = (2.0 * it + 1.0 - m) / m;
            const double c[3] = {1.0, cu, ct};
            const double cn = std::sqrt(1 + cu * cu + ct * ct);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const double u = (2.0 * (iu + a) - m) / m, t = (2.0 * (it + b) - m) / m;
                    const double q[3] = {1.0, u, t};
                    const double qn = std::sqrt(1 + u * u + t * t);
                    const double d = (c[0] * q[0] + c[1] * q[1] + c[2] * q[2]) / (cn * qn);
                    worst = std::max(worst, std::acos(std::min(1.0, d)));
                }
        }
    return worst;
}

LevelTemplate hf_template(const Plan &P, const LevelInfo &L)
{
    LevelTemplate T;
    T.hf = true;
    T.w = L.w;
    T.m = L.m;
    const double w = L.w, lam = P.lambda, k = P.k;
    const double rho = 1.05 * 0.5 * std::sqrt(3.0) * w;
    const int reach = (int)std::floor(P.opt.c_d * k * w + 1e-9) + 1;  // near if Chebyshev offset <= reach
    const double rc_min = (reach + 1) * w;                            // smallest interacting centre distance
    const double margin = std::asin(std::min(1.0, rho / rc_min));
    const double th = std::min(M_PI / 2, cell_angle(L.m) + 1.25 * margin + 0.02);
    const double r_in = rc_min - rho;
    const double r_out = std::max(16.0 * r_in, 4.0 * P.root_w);
    T.theta_cone = th;
    T.r_in = r_in;
    T.r_out = r_out;
    // check candidates: caps at log-spaced radii
    const double dth = lam / (6.0 * rho);
    const int ndir = std::min(4000, std::max(24, (int)std::ceil(2.0 * M_PI * (1.0 - std::cos(th)) / (dth * dth))));
    const int nr = 10;
    std::vector<double> Y;
    for (int q = 0; q < nr; ++q) {
        const double r = r_in * std::pow(r_out / r_in, (double)q / (nr - 1));
        cap_points(q == 0 ? 2 * ndir : ndir, th, r, Y);
    }
    // equivalent candidates: sphere of radius rho and two inner shells
    std::vector<double> Xc;
    const double shells[3] = {1.0, 0.7, 0.4};
    for (double f : shells) {
        const double rr = rho * f;
        const int n = std::max(16, (int)std::ceil(4.0 * M_PI * rr * rr / std::pow(lam / 5.0, 2)));
        cap_points(n, M_PI, rr, Xc);
    }
    const int ny = (int)Y.size() / 3, nxc = (int)Xc.size() / 3;
    // randomised column skeleton of A = G(Y, Xc): sketch B = Omega A
    const int ell = std::min(ny, 320);
    CMat Om = gaussian_sketch(ell, ny, 12345 + L.m);
    CMat Bsk(ell, nxc);
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = 0; j < nxc; ++j) {
        std::vector<cplx> col(ny);
        for (int i = 0; i < ny; ++i) col[i] = kernel_G(&Y[3 * i], &Xc[3 * j], k);
        for (int a = 0; a < ell; ++a) {
            cplx s = 0.0;
            for (int i = 0; i < ny; ++i) s += Om(a, i) * col[i];
            Bsk(a, j) = s;
        }
    }
    const double id_tol = 0.05 * svd_eps(P);
    std::vector<int> sel = select_columns(Bsk, id_tol, ell - 8);
    T.X.resize(3 * sel.size());
    for (size_t t = 0; t < sel.size(); ++t)
        for (int d = 0; d < 3; ++d) T.X[3 * t + d] = Xc[3 * sel[t] + d];
    T.Y = Y;
    finish_template(T, k, svd_eps(P));
    return T;
}

void rotate(const std::array<double, 9> &R, const std::vector<double> &in, std::vector<double> &out)
{
    const size_t n = in.size() / 3;
    out.resize(in.size());
    for (size_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            out[3 * i + a] = R[3 * a] * in[3 * i] + R[3 * a + 1] * in[3 * i + 1] + R[3 * a + 2] * in[3 * i + 2];
}

// Surface grid of the cube of half-width a with spacing at most h.
std::vector<double> cube_surface_spacing(double a, double h)
{
    return cube_surface(std::max(4, (int)std::ceil(2.0 * a / h) + 1), a);
}

// Uniform point on the surface of the cube of half-width a, from two
// uniform numbers in [0, 1) and a face index.
void cube_surface_point(double a, int face, double u, double v, double *p)
{
    const int ax = face >> 1;
    p[ax] = (face & 1) ? -a : a;
    p[(ax + 1) % 3] = a * (2.0 * u - 1.0);
    p[(ax + 2) % 3] = a * (2.0 * v - 1.0);
}

// Small deterministic generator for the sampling below (splitmix64).
struct Mix {
    uint64_t x;
    uint64_t next()
    {
        uint64_t z = (x += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    double uni() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
};

// Greedy pivoted selection of up to max_k rows of A (n x c), stopping at a
// relative residual of tol: the columns of A^T.
std::vector<int> select_rows(const CMat &A, double tol, int max_k)
{
    CMat At(A.n, A.m);
    for (int j = 0; j < A.n; ++j)
        for (int i = 0; i < A.m; ++i) At(j, i) = A(i, j);
    return select_columns(At, tol, max_k);
}

// High-frequency template of one wedge orbit (representative wedge zr of a
// level of width w).  The outgoing field of the cube's sources is needed
// only where the method evaluates it:
//  (a) M2L: at the equivalent points of the target cubes B, whose centre
//      offsets c_B - c_C are the level's operator offsets of this orbit
//      (section 3.1.1: same-level pairs outside the near field, in this
//      wedge), i.e. on the surfaces of the cubes at those offsets;
//  (b) M2M: at the check points of the parent's templates for the parent
//      wedges that nest in this wedge, seen from each of the eight child
//      positions.
// Check candidates sample (a) and take (b) whole.  Equivalent candidates
// are a grid on the cube's surface (half-width 1.05 w/2) that encloses the
// sources; the equivalent points are a column skeleton of the interaction
// matrix, the check points a row skeleton of what remains, both selected at
// tolerance 0.05 eps (the sampling of section 3.1.2 with controlling
// accuracy eps), and R = G(Y, X) is truncated by eq. eq_invr.
OrbitTemplate hf_orbit_template(const Plan &P, int l, int zr, const std::vector<double> &parent_checks)
{
    const LevelInfo &L = P.levels[l];
    const double w = L.w, lam = P.lambda, k = P.k;
    const double a = 1.05 * 0.5 * w;
    // candidate spacing lambda/5, coarser on wide cubes (at most ~4000 candidates)
    const std::vector<double> Xc = cube_surface_spacing(a, std::max(lam / 5.0, 2.0 * a * std::sqrt(6.0 / 4000.0)));
    const int nxc = (int)Xc.size() / 3;
    // (a) the operator offsets of this orbit (canonical frame, units of w)
    std::vector<std::array<int, 3>> offs;
    int omin = 1 << 30;
    for (const auto &ki : P.m2l_keyinfo[l])
        if (ki[0] == zr) {
            offs.push_back({ki[1], ki[2], ki[3]});
            omin = std::min(omin, std::max({std::abs(ki[1]), std::abs(ki[2]), std::abs(ki[3])}));
        }
    Mix rng{0x51ed2701ull + 977ull * (uint64_t)zr + 131ull * (uint64_t)l};
    std::vector<double> Ya;
    auto add_on_cube = [&](const std::array<int, 3> &o, int n) {
        for (int t = 0; t < n; ++t) {
            double p[3];
            cube_surface_point(a, (int)(rng.next() % 6), rng.uni(), rng.uni(), p);
            for (int d = 0; d < 3; ++d) Ya.push_back(o[d] * w + p[d]);
        }
    };
    if (!offs.empty()) {
        // a fixed budget shared by the offsets, at most what resolves one
        // target cube's surface at lambda/2.5; the nearest offsets, which bound
        // the accuracy, get at least 48 each
        const int budget = 24000;
        const int n_surf = std::max(16, (int)std::ceil(6.0 * std::pow(2.0 * a / (lam / 2.5), 2)));
        const int per = std::max(1, std::min(n_surf, budget / (int)offs.size()));
        for (const auto &o : offs) {
            const int cheb = std::max({std::abs(o[0]), std::abs(o[1]), std::abs(o[2])});
            add_on_cube(o, cheb == omin ? std::max(per, 48) : per);
        }
    }
    const int nya = (int)Ya.size() / 3, nyb = (int)parent_checks.size() / 3;
    std::vector<double> Yall(Ya);
    Yall.insert(Yall.end(), parent_checks.begin(), parent_checks.end());
    const int nyall = nya + nyb;
    if (nyall == 0) throw std::runtime_error("high-frequency template without evaluation points");
    // column skeleton on a subsample of the check candidates
    std::vector<int> sub;
    {
        const int want_a = std::min(nya, 3000), want_b = std::min(nyb, 1500);
        for (int t = 0; t < want_a; ++t) sub.push_back((int)((int64_t)t * nya / want_a));
        for (int t = 0; t < want_b; ++t) sub.push_back(nya + (int)((int64_t)t * nyb / want_b));
    }
    const int ns = (int)sub.size();
    const int ell = std::min(ns, 256);
    CMat Om = gaussian_sketch(ell, ns, 7777 + 31 * (uint64_t)zr + (uint64_t)l);
    CMat Bsk(ell, nxc);
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = 0; j < nxc; ++j) {
        std::vector<cplx> col(ns);
        for (int i = 0; i < ns; ++i) col[i] = kernel_G(&Yall[3 * (size_t)sub[i]], &Xc[3 * (size_t)j], k);
        for (int q = 0; q < ell; ++q) {
            cplx acc = 0.0;
            for (int i = 0; i < ns; ++i) acc += Om(q, i) * col[i];
            Bsk(q, j) = acc;
        }
    }
    const double id_tol = 0.05 * hf_svd_eps(P);
    const std::vector<int> xs = select_columns(Bsk, id_tol, ell - 8);
    const int nx = (int)xs.size();
    OrbitTemplate T;
    T.X.resize(3 * (size_t)nx);
    for (int t = 0; t < nx; ++t)
        for (int d = 0; d < 3; ++d) T.X[3 * t + d] = Xc[3 * (size_t)xs[t] + d];
    // row skeleton of G(all check candidates, X)
    CMat A(nyall, nx);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nyall; ++i)
        for (int j = 0; j < nx; ++j) A(i, j) = kernel_G(&Yall[3 * (size_t)i], &T.X[3 * (size_t)j], k);
    std::vector<int> ys = select_rows(A, id_tol, nx);
    // oversample: as many again spread over the candidates, so that R is
    // fitted in the least-squares sense rather than interpolated
    {
        std::vector<char> taken(nyall, 0);
        for (int i : ys) taken[i] = 1;
        const int extra = std::min((int)ys.size(), nyall - (int)ys.size());
        for (int t = 0, added = 0; added < extra && t < 4 * nyall; ++t) {
            const int i = (int)(rng.next() % (uint64_t)nyall);
            if (!taken[i]) {
                taken[i] = 1;
                ys.push_back(i);
                ++added;
            }
        }
    }
    T.Y.resize(3 * ys.size());
    for (size_t t = 0; t < ys.size(); ++t)
        for (int d = 0; d < 3; ++d) T.Y[3 * t + d] = Yall[3 * (size_t)ys[t] + d];
    return T;
}

// R = G(Y, X) = U S V^H of an orbit template, truncated at eps (eq. eq_invr)
// and padded with zero basis vectors up to the level's common dimension s.
void finish_orbit(OrbitTemplate &T, double k, double eps)
{
    const int ny = (int)T.Y.size() / 3, nx = (int)T.X.size() / 3;
    CMat R(ny, nx);
    for (int j = 0; j < nx; ++j)
        for (int i = 0; i < ny; ++i) R(i, j) = kernel_G(&T.Y[3 * i], &T.X[3 * j], k);
    SVD d = svd(R);
    T.sing = d.s;
    T.rank = std::max(1, truncation_rank(d.s, eps));
    // Vt and W are filled once the level's s is known
    T.Vt = d.V;
    T.W = d.U;
}

void pad_orbit(OrbitTemplate &T, int s)
{
    const int ny = (int)T.Y.size() / 3, nx = (int)T.X.size() / 3;
    CMat V(nx, s), W(s, ny);
    for (int c = 0; c < T.rank; ++c) {
        for (int i = 0; i < nx; ++i) V(i, c) = T.Vt(i, c);
        for (int i = 0; i < ny; ++i) W(c, i) = std::conj(T.W(i, c)) / T.sing[c];
    }
    T.Vt = std::move(V);
    T.W = std::move(W);
}

int64_t push_matrix(Plan &P, const CMat &A)
{
    const int64_t off = (int64_t)P.matpool.size();
    P.matpool.insert(P.matpool.end(), A.a.begin(), A.a.end());
    return off;
}

}  // namespace

void build_templates(Plan &P)
{
    const int nlev = (int)P.levels.size();
    P.tmpl.assign(nlev, LevelTemplate());
    std::vector<int> needed;
    for (int l = 0; l < nlev; ++l) {
        const LevelInfo &L = P.levels[l];
        if (L.n_out + L.n_in > 0) needed.push_back(l);
    }
    // low-frequency templates are independent of each other: one level per thread
    std::vector<int> lf_levels;
    for (int l : needed)
        if (!P.levels[l].hf) lf_levels.push_back(l);
#pragma omp parallel for schedule(dynamic, 1)
    for (size_t q = 0; q < lf_levels.size(); ++q) P.tmpl[lf_levels[q]] = lf_template(P, P.levels[lf_levels[q]].w);
    // top-down: a high-frequency template samples its parent's check points
    for (int l : needed) {
        const LevelInfo &L = P.levels[l];
        if (!L.hf) continue;
        LevelTemplate &T = P.tmpl[l];
        T.hf = true;
        T.w = L.w;
        T.m = L.m;
        // orbits of the wedges that carry slots at this level
        std::vector<int> orbits;
        {
            std::vector<char> used(L.nwedge, 0);
            for (size_t t = 0; t < L.out_slot.size(); ++t)
                if (L.out_slot[t] >= 0 || L.in_slot[t] >= 0) used[t % L.nwedge] = 1;
            std::vector<char> seen(L.nwedge, 0);
            for (int z = 0; z < L.nwedge; ++z)
                if (used[z] && !seen[L.frames[z].orbit]) {
                    seen[L.frames[z].orbit] = 1;
                    orbits.push_back(L.frames[z].orbit);
                }
        }
        if (P.opt.hf_template == 1) {
            // earlier construction: one +x template rotated to each orbit
            LevelTemplate H = hf_template(P, L);
            if (P.opt.original) to_original_basis(H.Vt, H.W, H.s, (int)H.X.size() / 3);
            T.s = H.s;
            T.theta_cone = H.theta_cone;
            T.r_in = H.r_in;
            T.r_out = H.r_out;
            for (int zr : orbits) {
                OrbitTemplate O;
                rotate(L.frames[zr].R, H.X, O.X);
                rotate(L.frames[zr].R, H.Y, O.Y);
                O.Vt = H.Vt;
                O.W = H.W;
                O.sing = H.sing;
                O.rank = H.s;
                T.orbit.emplace(zr, std::move(O));
            }
        } else {
            const bool parent_hf = l > 0 && P.levels[l - 1].hf && P.tmpl[l - 1].hf && !P.tmpl[l - 1].orbit.empty();
            std::vector<OrbitTemplate> built(orbits.size());
#pragma omp parallel for schedule(dynamic, 1) if (orbits.size() > 1)
            for (size_t q = 0; q < orbits.size(); ++q) {
                const int zr = orbits[q];
                std::vector<double> pc;
                if (parent_hf) {
                    // parent wedges nested in zr, their check points seen from the eight child centres
                    const LevelInfo &Lp = P.levels[l - 1];
                    const LevelTemplate &Tp = P.tmpl[l - 1];
                    for (int zp = 0; zp < Lp.nwedge; ++zp) {
                        if (wedge_child(zp, Lp.m) != zr) continue;
                        auto it = Tp.orbit.find(Lp.frames[zp].orbit);
                        if (it == Tp.orbit.end()) continue;
                        std::vector<double> Yp;
                        rotate(Lp.frames[zp].G, it->second.Y, Yp);
                        for (int oct = 0; oct < 8; ++oct) {
                            const double off[3] = {((oct & 1) - 0.5) * L.w, (((oct >> 1) & 1) - 0.5) * L.w,
                                                   (((oct >> 2) & 1) - 0.5) * L.w};
                            for (size_t t = 0; t < Yp.size() / 3; ++t)
                                for (int d = 0; d < 3; ++d) pc.push_back(Yp[3 * t + d] - off[d]);
                        }
                    }
                }
                built[q] = hf_orbit_template(P, l, zr, pc);
                finish_orbit(built[q], P.k, hf_svd_eps(P));
            }
            int s = 0;
            for (const OrbitTemplate &O : built) s = std::max(s, O.rank);
            T.s = s;
            int s_orig = 0;
            for (const OrbitTemplate &O : built) s_orig = std::max(s_orig, (int)O.X.size() / 3);
            for (size_t q = 0; q < orbits.size(); ++q) {
                pad_orbit(built[q], s);
                if (P.opt.original) {
                    int so = s;
                    to_original_basis(built[q].Vt, built[q].W, so, (int)built[q].X.size() / 3, s_orig);
                }
                T.orbit.emplace(orbits[q], std::move(built[q]));
            }
            if (P.opt.original) T.s = s_orig;
        }
        for (const auto &kv : T.orbit) {
            T.n_equiv_max = std::max(T.n_equiv_max, (int)kv.second.X.size() / 3);
            T.n_check_max = std::max(T.n_check_max, (int)kv.second.Y.size() / 3);
        }
        if (P.opt.verbose) {
            std::fprintf(stderr, "[fdbem] level w = %.4g: %zu wedge orbits, s = %d (equivalent <= %d, check <= %d)\n",
                         L.w, T.orbit.size(), T.s, T.n_equiv_max, T.n_check_max);
            std::fflush(stderr);
        }
    }
    P.max_s = 0;
    P.max_Y = 0;
    for (int l : needed) {
        P.max_s = std::max(P.max_s, P.tmpl[l].s);
        P.max_Y = std::max(P.max_Y, (int)P.tmpl[l].Y.size() / 3);
    }
}

void build_operators(Plan &P)
{
    const int nlev = (int)P.levels.size();
    P.matpool.clear();
    // density layout
    int64_t ob = 0, ib = 0;
    for (int l = 0; l < nlev; ++l) {
        LevelInfo &L = P.levels[l];
        L.out_base = ob;
        L.in_base = ib;
        ob += (int64_t)L.n_out * P.tmpl[l].s;
        ib += (int64_t)L.n_in * P.tmpl[l].s;
    }
    P.out_total = ob;
    P.in_total = ib;

    // ---- M2L operators per level
    P.m2l_lists.assign(nlev, GemvList());
    for (int l = 0; l < nlev; ++l) {
        const LevelInfo &L = P.levels[l];
        const int nk = P.m2l_nkeys[l];
        if (nk == 0) continue;
        const LevelTemplate &T = P.tmpl[l];
        const int s = T.s;
        std::vector<CMat> dense(nk), Uf(nk), Vf(nk);
        std::vector<int> rk(nk, -1);
        const double leps = lr_eps(P);
        // low-rank M2L (section 4.2) unless disabled (lowrank_eps < 0) or the
        // original method is requested
        const bool use_lowrank = !P.opt.original && P.opt.lowrank_eps >= 0;
        std::atomic<int> done{0};
        const auto t_lev = std::chrono::steady_clock::now();
        auto last = t_lev;
#pragma omp parallel for schedule(dynamic, 4)
        for (int key = 0; key < nk; ++key) {
            if (P.opt.verbose) {
                // a progress line about every 30 s on long levels
                const int d = done.fetch_add(1) + 1;
#pragma omp critical(fdbem_progress)
                {
                    const auto now = std::chrono::steady_clock::now();
                    if (std::chrono::duration<double>(now - last).count() > 30.0) {
                        last = now;
                        std::fprintf(stderr, "[fdbem] M2L operators of level %d: %d of %d (%.0f s)\n", l, d, nk,
                                     std::chrono::duration<double>(now - t_lev).count());
                        std::fflush(stderr);
                    }
                }
            }
            const auto &ki = P.m2l_keyinfo[l][key];
            std::vector<double> Xb, Xa;  // source (C) and target (B) equivalent points
            double off[3] = {ki[1] * L.w, ki[2] * L.w, ki[3] * L.w};
            // the canonical offset lies in the orbit's representative wedge, whose
            // template is in that frame; the target's incoming points are the
            // reflection (a signed permutation, so again a template of the orbit)
            const CMat &Vt = L.hf ? T.orbit.at(ki[0]).Vt : T.Vt;
            if (L.hf) {
                Xb = T.orbit.at(ki[0]).X;
                Xa.resize(Xb.size());
                for (size_t t = 0; t < Xb.size() / 3; ++t)
                    for (int d = 0; d < 3; ++d) Xa[3 * t + d] = off[d] - Xb[3 * t + d];
            } else {
                Xb = T.X;
                Xa.resize(Xb.size());
                for (size_t t = 0; t < Xb.size() / 3; ++t)
                    for (int d = 0; d < 3; ++d) Xa[3 * t + d] = off[d] + Xb[3 * t + d];
            }
            const int nx = (int)Xb.size() / 3;
            CMat K(nx, nx);
            for (int j = 0; j < nx; ++j)
                for (int i = 0; i < nx; ++i) K(i, j) = kernel_G(&Xa[3 * i], &Xb[3 * j], P.k);
            CMat KV = matmul(K, 'N', Vt, 'N');
            CMat Kt = matmul(Vt, 'T', KV, 'N');  // s x s
            // low rank when the eps-rank r is below s/2 (strict, section 4.2)
            CMat U, V;
            int r = 0;
            if (use_lowrank && lowrank_factor(Kt, leps, (s - 1) / 2, 0x9e37ull * (uint64_t)(key + 1) + (uint64_t)l, U, V, r)) {
                Uf[key] = std::move(U);
                Vf[key] = std::move(V);
                rk[key] = r;
            } else {
                dense[key] = std::move(Kt);
            }
        }
        std::vector<int64_t> key_off(nk);
        for (int key = 0; key < nk; ++key) {
            if (rk[key] >= 0) {
                key_off[key] = push_matrix(P, Uf[key]);
                push_matrix(P, Vf[key]);
            } else
                key_off[key] = push_matrix(P, dense[key]);
        }
        GemvList &G = P.m2l_lists[l];
        G.rows = G.cols = s;
        std::vector<int> slot_wedge(L.n_in, 0);
        for (size_t t = 0; t < L.in_slot.size(); ++t)
            if (L.in_slot[t] >= 0) slot_wedge[L.in_slot[t]] = (int)(t % L.nwedge);
        G.ptr.push_back(0);
        const auto &V = P.m2l[l];
        for (size_t q = 0; q < V.size(); ++q) {
            if (q == 0 || V[q].tgt_slot != V[q - 1].tgt_slot) {
                if (q > 0) G.ptr.push_back((int)G.in_off.size());
                G.out_off.push_back(L.in_base + (int64_t)V[q].tgt_slot * s);
                G.out_wedge.push_back(slot_wedge[V[q].tgt_slot]);
            }
            G.in_off.push_back(L.out_base + (int64_t)V[q].src_slot * s);
            G.mat_off.push_back(key_off[V[q].key]);
            G.rank.push_back(rk[V[q].key]);
        }
        if (!V.empty()) G.ptr.push_back((int)G.in_off.size());
    }

    // ---- M2M (upward) and L2L (downward) between level l (parent) and l+1
    P.m2m_lists.assign(nlev, GemvList());
    P.l2l_lists.assign(nlev, GemvList());
    for (int l = 0; l + 1 < nlev; ++l) {
        const LevelInfo &Lp = P.levels[l], &Lc = P.levels[l + 1];
        const LevelTemplate &Tp = P.tmpl[l], &Tc = P.tmpl[l + 1];
        if (Lp.n_out + Lp.n_in == 0) continue;
        // collect the (parent wedge, octant) operators needed
        std::map<std::pair<int, int>, int64_t> mats;
        auto need = [&](int zp, int oct) { mats.emplace(std::make_pair(zp, oct), -1); };
        for (size_t a = 0; a < Lp.cubes.size(); ++a) {
            const Cube &Par = P.cubes[Lp.cubes[a]];
            for (int zp = 0; zp < Lp.nwedge; ++zp) {
                const bool po = Lp.out_slot[a * Lp.nwedge + zp] >= 0;
                const bool pi = Lp.in_slot[a * Lp.nwedge + zp] >= 0;
                if (!po && !pi) continue;
                for (int o = 0; o < 8; ++o)
                    if (Par.child[o] >= 0) need(zp, o);
            }
        }
        std::vector<std::pair<int, int>> keys;
        for (auto &kv : mats) keys.push_back(kv.first);
        std::vector<CMat> Ms(keys.size());
#pragma omp parallel for schedule(dynamic, 4)
        for (size_t q = 0; q < keys.size(); ++q) {
            const int zp = keys[q].first, oct = keys[q].second;
            std::vector<double> Yp, Xc;
            const CMat *Wp = &Tp.W, *Vc = &Tc.Vt;
            if (Lp.hf) {
                const OrbitTemplate &O = Tp.orbit.at(Lp.frames[zp].orbit);
                rotate(Lp.frames[zp].G, O.Y, Yp);
                Wp = &O.W;
            } else
                Yp = Tp.Y;
            const int zc = Lc.hf ? wedge_child(zp, Lp.m) : 0;
            if (Lc.hf) {
                const OrbitTemplate &O = Tc.orbit.at(Lc.frames[zc].orbit);
                rotate(Lc.frames[zc].G, O.X, Xc);
                Vc = &O.Vt;
            } else
                Xc = Tc.X;
            const double wc = Lc.w;
            const double off[3] = {((oct & 1) - 0.5) * wc, (((oct >> 1) & 1) - 0.5) * wc, (((oct >> 2) & 1) - 0.5) * wc};
            for (size_t t = 0; t < Xc.size() / 3; ++t)
                for (int d = 0; d < 3; ++d) Xc[3 * t + d] += off[d];
            const int ny = (int)Yp.size() / 3, nx = (int)Xc.size() / 3;
            CMat E(ny, nx);
            for (int j = 0; j < nx; ++j)
                for (int i = 0; i < ny; ++i) E(i, j) = kernel_G(&Yp[3 * i], &Xc[3 * j], P.k);
            CMat EV = matmul(E, 'N', *Vc, 'N');
            Ms[q] = matmul(*Wp, 'N', EV, 'N');  // s_p x s_c
        }
        for (size_t q = 0; q < keys.size(); ++q) mats[keys[q]] = push_matrix(P, Ms[q]);
        // upward list: parent out slots
        GemvList &U = P.m2m_lists[l];
        U.rows = Tp.s;
        U.cols = Tc.s;
        U.ptr.push_back(0);
        // downward list: child in slots
        GemvList &D = P.l2l_lists[l + 1];
        D.rows = Tc.s;
        D.cols = Tp.s;
        D.trans = 1;
        D.ptr.push_back(0);
        for (size_t a = 0; a < Lp.cubes.size(); ++a) {
            const Cube &Par = P.cubes[Lp.cubes[a]];
            for (int zp = 0; zp < Lp.nwedge; ++zp) {
                const int so = Lp.out_slot[a * Lp.nwedge + zp];
                if (so < 0) continue;
                const int zc = Lc.hf ? wedge_child(zp, Lp.m) : 0;
                U.out_off.push_back(Lp.out_base + (int64_t)so * Tp.s);
                for (int o = 0; o < 8; ++o) {
                    if (Par.child[o] < 0) continue;
                    const Cube &Ch = P.cubes[Par.child[o]];
                    const int cs = Lc.out_slot[(size_t)Ch.local * Lc.nwedge + zc];
                    if (cs < 0) throw std::runtime_error("missing child outgoing slot");
                    U.in_off.push_back(Lc.out_base + (int64_t)cs * Tc.s);
                    U.mat_off.push_back(mats[{zp, o}]);
                    U.rank.push_back(-1);
                }
                U.ptr.push_back((int)U.in_off.size());
            }
        }
        // child in slots: gather parent wedges that map into them
        for (size_t a = 0; a < Lc.cubes.size(); ++a) {
            const Cube &Ch = P.cubes[Lc.cubes[a]];
            if (Ch.parent < 0) continue;
            const Cube &Par = P.cubes[Ch.parent];
            int oct = -1;
            for (int o = 0; o < 8; ++o)
                if (Par.child[o] == Lc.cubes[a]) oct = o;
            for (int zc = 0; zc < Lc.nwedge; ++zc) {
                const int si = Lc.in_slot[a * Lc.nwedge + zc];
                if (si < 0) continue;
                std::vector<std::pair<int64_t, int64_t>> ent;
                for (int zp = 0; zp < Lp.nwedge; ++zp) {
                    const int ps = Lp.in_slot[(size_t)Par.local * Lp.nwedge + zp];
                    if (ps < 0) continue;
                    const int zcc = Lc.hf ? wedge_child(zp, Lp.m) : 0;
                    if (zcc != zc) continue;
                    ent.push_back({Lp.in_base + (int64_t)ps * Tp.s, mats[{zp, oct}]});
                }
                if (ent.empty()) continue;
                D.out_off.push_back(Lc.in_base + (int64_t)si * Tc.s);
                for (auto &e : ent) {
                    D.in_off.push_back(e.first);
                    D.mat_off.push_back(e.second);
                    D.rank.push_back(-1);
                }
                D.ptr.push_back((int)D.in_off.size());
            }
        }
    }

    // ---- leaf tasks
    P.s2m_tasks.clear();
    P.l2t_tasks.clear();
    P.max_Y_leaf = 0;
    for (int id : P.leaves) {
        const Cube &c = P.cubes[id];
        const LevelInfo &L = P.levels[c.level];
        if (L.hf) {
            bool any = false;
            for (int z = 0; z < L.nwedge; ++z)
                any |= L.out_slot[(size_t)c.local * L.nwedge + z] >= 0 || L.in_slot[(size_t)c.local * L.nwedge + z] >= 0;
            if (any) throw std::runtime_error("high-frequency leaves are not supported by this leaf rule");
            continue;
        }
        const int so = L.out_slot[c.local], si = L.in_slot[c.local];
        const int s = P.tmpl[c.level].s;
        LeafTask t;
        t.start = c.start;
        t.end = c.end;
        t.tmpl = c.level;
        for (int d = 0; d < 3; ++d) t.center[d] = P.root_center[d] - 0.5 * P.root_w + (c.ijk[d] + 0.5) * L.w;
        if (so >= 0) {
            t.slot_off = L.out_base + (int64_t)so * s;
            P.s2m_tasks.push_back(t);
        }
        if (si >= 0) {
            t.slot_off = L.in_base + (int64_t)si * s;
            P.l2t_tasks.push_back(t);
        }
        if (so >= 0 || si >= 0) P.max_Y_leaf = std::max(P.max_Y_leaf, (int)P.tmpl[c.level].Y.size() / 3);
    }
}

}  // namespace fdbem

namespace fdbem {

void build_m2l_tiles(Plan &P, int tile, int chunk)
{
    const int nlev = (int)P.levels.size();
    P.m2l_tiles.assign(nlev, M2LTiles());
    for (int l = 0; l < nlev; ++l) {
        const GemvList &G = P.m2l_lists[l];
        M2LTiles &T = P.m2l_tiles[l];
        T.tile = tile;
        T.chunk = chunk;
        T.s = G.rows;
        const int n_out = (int)G.out_off.size();
        if (n_out == 0) continue;
        std::vector<int> order(n_out);
        for (int t = 0; t < n_out; ++t) order[t] = t;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return G.out_wedge[a] < G.out_wedge[b]; });
        T.tgt_off.resize(n_out);
        for (int t = 0; t < n_out; ++t) T.tgt_off[t] = G.out_off[order[t]];
        struct E {
            int64_t mat;
            int rank, tl;
            int64_t src;
        };
        std::vector<E> es, rest;
        std::vector<char> used(tile, 0);
        for (int t0 = 0; t0 < n_out; t0 += tile) {
            const int nt = std::min(tile, n_out - t0);
            es.clear();
            for (int t = 0; t < nt; ++t)
                for (int e = G.ptr[order[t0 + t]]; e < G.ptr[order[t0 + t] + 1]; ++e)
                    es.push_back({G.mat_off[e], G.rank[e], t, G.in_off[e]});
            // group by operator; runs split into chunks with distinct targets
            std::stable_sort(es.begin(), es.end(), [](const E &a, const E &b) { return a.mat < b.mat; });
            T.tile_ntgt.push_back(nt);
            T.tile_cptr.push_back((int)T.ch_mat.size());
            size_t i = 0;
            while (i < es.size()) {
                size_t j = i;
                while (j < es.size() && es[j].mat == es[i].mat) ++j;
                std::vector<E> pending(es.begin() + i, es.begin() + j);
                while (!pending.empty()) {
                    rest.clear();
                    std::fill(used.begin(), used.end(), 0);
                    int cnt = 0;
                    T.ch_mat.push_back(pending[0].mat);
                    T.ch_rank.push_back(pending[0].rank);
                    T.ch_pptr.push_back((int)T.pr_tl.size());
                    for (const E &x : pending) {
                        if (cnt < chunk && !used[x.tl]) {
                            used[x.tl] = 1;
                            T.pr_tl.push_back(x.tl);
                            T.pr_src.push_back(x.src);
                            ++cnt;
                        } else
                            rest.push_back(x);
                    }
                    pending.swap(rest);
                }
                i = j;
            }
        }
        T.tile_cptr.push_back((int)T.ch_mat.size());
        T.ch_pptr.push_back((int)T.pr_tl.size());
        for (int r : T.ch_rank) T.max_rank = std::max(T.max_rank, r);
    }
}

}  // namespace fdbem

namespace fdbem {

static M2LChunks build_chunks_range(const GemvList &G, int chunk, int o0, int o1)
{
    M2LChunks C;
    C.chunk = chunk;
    C.s = G.rows;
    C.cols = G.cols;
    C.trans = G.trans;
    if (o1 <= o0) return C;
    const int64_t e0 = G.ptr[o0], e1 = G.ptr[o1], ne = e1 - e0;
    std::vector<int64_t> tgt(ne);
    for (int o = o0; o < o1; ++o) {
        C.red_out.push_back(G.out_off[o]);
        C.red_ptr.push_back(G.ptr[o] - e0);
        for (int e = G.ptr[o]; e < G.ptr[o + 1]; ++e) tgt[e - e0] = G.out_off[o];
    }
    C.red_ptr.push_back(ne);
    std::vector<int64_t> idx(ne);
    for (int64_t e = 0; e < ne; ++e) idx[e] = e;
    // by operator, then by target (nearby targets share cache lines)
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        const int64_t ma = G.mat_off[e0 + a], mb = G.mat_off[e0 + b];
        return ma != mb ? ma < mb : tgt[a] < tgt[b];
    });
    C.pr_tgt.resize(ne);
    C.pr_src.resize(ne);
    C.pr_pos.resize(ne);
    for (int64_t q = 0; q < ne; ++q) {
        const int64_t e = idx[q];
        const int64_t mat = G.mat_off[e0 + e];
        if (q == 0 || mat != G.mat_off[e0 + idx[q - 1]] || (q - C.ch_pptr.back()) >= chunk) {
            C.ch_mat.push_back(mat);
            C.ch_rank.push_back(G.rank[e0 + e]);
            C.ch_pptr.push_back((int)q);
        }
        C.pr_tgt[q] = tgt[e];
        C.pr_src[q] = G.in_off[e0 + e];
        C.pr_pos[q] = e;
    }
    C.ch_pptr.push_back((int)ne);
    for (int r : C.ch_rank) C.max_rank = std::max(C.max_rank, r);
    return C;
}

M2LChunks build_chunks(const GemvList &G, int chunk)
{
    return build_chunks_range(G, chunk, 0, (int)G.out_off.size());
}

std::vector<M2LChunks> build_chunk_slabs(const GemvList &G, int chunk, int64_t max_entries)
{
    std::vector<M2LChunks> out;
    const int n_out = (int)G.out_off.size();
    int o0 = 0;
    while (o0 < n_out) {
        int o1 = o0 + 1;
        while (o1 < n_out && (int64_t)G.ptr[o1 + 1] - G.ptr[o0] <= max_entries) ++o1;
        out.push_back(build_chunks_range(G, chunk, o0, o1));
        o0 = o1;
    }
    return out;
}

void build_m2l_chunks(Plan &P, int chunk)
{
    const int nlev = (int)P.levels.size();
    P.m2l_chunks.assign(nlev, M2LChunks());
    for (int l = 0; l < nlev; ++l) P.m2l_chunks[l] = build_chunks(P.m2l_lists[l], chunk);
}

}  // namespace fdbem
