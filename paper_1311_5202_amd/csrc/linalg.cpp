#include "linalg.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace fdbem {

CMat matmul(const CMat &A, char opA, const CMat &B, char opB)
{
    const int am = (opA == 'N') ? A.m : A.n;
    const int ak = (opA == 'N') ? A.n : A.m;
    const int bk = (opB == 'N') ? B.m : B.n;
    const int bn = (opB == 'N') ? B.n : B.m;
    (void)bk;
    CMat C(am, bn);
    auto a_at = [&](int i, int l) -> cplx {
        if (opA == 'N') return A(i, l);
        if (opA == 'T') return A(l, i);
        return std::conj(A(l, i));
    };
    auto b_at = [&](int l, int j) -> cplx {
        if (opB == 'N') return B(l, j);
        if (opB == 'T') return B(j, l);
        return std::conj(B(j, l));
    };
    if (opA == 'N' && opB == 'N') {
        for (int j = 0; j < bn; ++j)
            for (int l = 0; l < ak; ++l) {
                const cplx b = B(l, j);
                const cplx *ac = A.col(l);
                cplx *cc = C.col(j);
                for (int i = 0; i < am; ++i) cc[i] += ac[i] * b;
            }
        return C;
    }
    if (opA != 'N' && opB == 'N') {
        // C(i,j) = sum_l op(A)(i,l) B(l,j): columns of A are contiguous
        for (int j = 0; j < bn; ++j)
            for (int i = 0; i < am; ++i) {
                const cplx *ac = A.col(i);
                const cplx *bc = B.col(j);
                cplx s = 0.0;
                if (opA == 'C')
                    for (int l = 0; l < ak; ++l) s += std::conj(ac[l]) * bc[l];
                else
                    for (int l = 0; l < ak; ++l) s += ac[l] * bc[l];
                C(i, j) = s;
            }
        return C;
    }
    for (int j = 0; j < bn; ++j)
        for (int i = 0; i < am; ++i) {
            cplx s = 0.0;
            for (int l = 0; l < ak; ++l) s += a_at(i, l) * b_at(l, j);
            C(i, j) = s;
        }
    return C;
}

static SVD svd_tall(const CMat &A)
{
    // one-sided (Hestenes) Jacobi: orthogonalise the columns of W = A V
    const int m = A.m, n = A.n;
    CMat W = A;
    CMat V(n, n);
    for (int i = 0; i < n; ++i) V(i, i) = 1.0;
    const double tol = 1e-15;
    // a rotation whose coupling is below rounding of the whole matrix changes
    // nothing that matters: skipping it lets columns at the noise level (a
    // numerically rank-deficient A) stop rotating instead of running every sweep
    double fro2 = 0.0;
    for (const cplx &v : A.a) fro2 += std::norm(v);
    const double negligible = 1e-32 * fro2;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int j = 0; j < n - 1; ++j)
            for (int k = j + 1; k < n; ++k) {
                cplx *wj = W.col(j), *wk = W.col(k);
                double al = 0.0, be = 0.0;
                cplx ga = 0.0;
                for (int i = 0; i < m; ++i) {
                    al += std::norm(wj[i]);
                    be += std::norm(wk[i]);
                    ga += std::conj(wj[i]) * wk[i];
                }
                const double ag = std::abs(ga);
                if (ag == 0.0 || ag <= tol * std::sqrt(al * be) || ag <= negligible) continue;
                off = std::max(off, ag / std::sqrt(al * be));
                const cplx ph = std::conj(ga) / ag;  // e^{-i phi}
                const double zeta = (be - al) / (2.0 * ag);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < m; ++i) {
                    const cplx a = wj[i], b = ph * wk[i];
                    wj[i] = c * a - s * b;
                    wk[i] = s * a + c * b;
                }
                cplx *vj = V.col(j), *vk = V.col(k);
                for (int i = 0; i < n; ++i) {
                    const cplx a = vj[i], b = ph * vk[i];
                    vj[i] = c * a - s * b;
                    vk[i] = s * a + c * b;
                }
            }
        if (off < tol) break;
    }
    std::vector<double> sv(n);
    for (int j = 0; j < n; ++j) {
        double s2 = 0.0;
        for (int i = 0; i < m; ++i) s2 += std::norm(W(i, j));
        sv[j] = std::sqrt(s2);
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return sv[a] > sv[b]; });
    SVD out;
    out.U = CMat(m, n);
    out.V = CMat(n, n);
    out.s.resize(n);
    for (int c = 0; c < n; ++c) {
        const int j = ord[c];
        out.s[c] = sv[j];
        const double inv = sv[j] > 0 ? 1.0 / sv[j] : 0.0;
        for (int i = 0; i < m; ++i) out.U(i, c) = W(i, j) * inv;
        for (int i = 0; i < n; ++i) out.V(i, c) = V(i, j);
    }
    return out;
}

SVD svd(const CMat &A)
{
    if (A.m >= A.n) return svd_tall(A);
    // wide: A^H = U' S V'^H  =>  A = V' S U'^H
    CMat AH(A.n, A.m);
    for (int j = 0; j < A.n; ++j)
        for (int i = 0; i < A.m; ++i) AH(j, i) = std::conj(A(i, j));
    SVD t = svd_tall(AH);
    SVD out;
    out.s = t.s;
    out.U = t.V;
    out.V = t.U;
    // only the first min(m,n) = A.m columns are meaningful
    return out;
}

int truncation_rank(const std::vector<double> &s, double eps)
{
    if (s.empty() || s[0] <= 0.0) return 0;
    int r = 0;
    for (double v : s)
        if (v >= eps * s[0]) ++r;
    return r;
}

std::vector<int> select_columns(const CMat &A, double tol, int max_k)
{
    const int m = A.m, n = A.n;
    CMat W = A;
    std::vector<double> nrm(n);
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += std::norm(W(i, j));
        nrm[j] = s;
    }
    std::vector<char> used(n, 0);
    std::vector<int> sel;
    double first = -1.0;
    std::vector<cplx> q(m);
    for (int it = 0; it < std::min({max_k, m, n}); ++it) {
        int p = -1;
        double best = -1.0;
        for (int j = 0; j < n; ++j)
            if (!used[j] && nrm[j] > best) {
                best = nrm[j];
                p = j;
            }
        if (p < 0) break;
        // recompute the pivot's norm exactly (the running update drifts)
        double pn = 0.0;
        for (int i = 0; i < m; ++i) pn += std::norm(W(i, p));
        pn = std::sqrt(pn);
        if (first < 0) first = pn;
        if (pn <= tol * first || pn == 0.0) break;
        used[p] = 1;
        sel.push_back(p);
        for (int i = 0; i < m; ++i) q[i] = W(i, p) / pn;
        for (int j = 0; j < n; ++j) {
            if (used[j]) continue;
            cplx *wj = W.col(j);
            cplx d = 0.0;
            for (int i = 0; i < m; ++i) d += std::conj(q[i]) * wj[i];
            double s = 0.0;
            for (int i = 0; i < m; ++i) {
                wj[i] -= d * q[i];
                s += std::norm(wj[i]);
            }
            nrm[j] = s;
        }
    }
    return sel;
}

static uint64_t splitmix(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

CMat gaussian_sketch(int k, int m, uint64_t seed)
{
    CMat S(k, m);
    uint64_t st = seed;
    const double sc = 1.0 / std::sqrt((double)k);
    for (size_t t = 0; t < S.a.size(); ++t) {
        double u1 = ((splitmix(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        double u2 = ((splitmix(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        double r = std::sqrt(-2.0 * std::log(u1));
        S.a[t] = cplx(r * std::cos(2 * M_PI * u2), r * std::sin(2 * M_PI * u2)) * sc;
    }
    return S;
}

void orthonormalize(CMat &A)
{
    const int m = A.m, n = A.n;
    for (int j = 0; j < n; ++j) {
        cplx *aj = A.col(j);
        double n0 = 0.0;
        for (int i = 0; i < m; ++i) n0 += std::norm(aj[i]);
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < j; ++q) {
                const cplx *aq = A.col(q);
                cplx d = 0.0;
                for (int i = 0; i < m; ++i) d += std::conj(aq[i]) * aj[i];
                for (int i = 0; i < m; ++i) aj[i] -= d * aq[i];
            }
        double nr = 0.0;
        for (int i = 0; i < m; ++i) nr += std::norm(aj[i]);
        if (!(nr > 1e-28 * n0) || nr == 0.0) {
            // dependent column: take the coordinate vector least covered so far
            for (int e = 0; e < m; ++e) {
                for (int i = 0; i < m; ++i) aj[i] = i == e ? 1.0 : 0.0;
                for (int pass = 0; pass < 2; ++pass)
                    for (int q = 0; q < j; ++q) {
                        const cplx *aq = A.col(q);
                        cplx d = 0.0;
                        for (int i = 0; i < m; ++i) d += std::conj(aq[i]) * aj[i];
                        for (int i = 0; i < m; ++i) aj[i] -= d * aq[i];
                    }
                nr = 0.0;
                for (int i = 0; i < m; ++i) nr += std::norm(aj[i]);
                if (nr > 0.25) break;
            }
        }
        const double inv = 1.0 / std::sqrt(nr);
        for (int i = 0; i < m; ++i) aj[i] *= inv;
    }
}

bool lowrank_factor(const CMat &A, double eps, int max_r, uint64_t seed, CMat &U, CMat &V, int &r)
{
    const int m = A.m, n = A.n;
    const int ell = std::min(std::min(m, n), max_r + 8);
    if (ell <= 0) return false;
    // range of A from A (A^H A) Omega, orthonormalised between the products
    CMat Om = gaussian_sketch(n, ell, seed);  // n x ell
    CMat Y = matmul(A, 'N', Om, 'N');         // m x ell
    orthonormalize(Y);
    CMat Z = matmul(A, 'C', Y, 'N');          // n x ell
    orthonormalize(Z);
    CMat Q = matmul(A, 'N', Z, 'N');          // m x ell
    orthonormalize(Q);
    CMat B = matmul(Q, 'C', A, 'N');          // ell x n
    SVD d = svd(B);
    r = truncation_rank(d.s, eps);
    if (r > max_r || r >= ell) return false;
    r = std::max(r, 1);
    U = CMat(m, r);
    V = CMat(r, n);
    for (int c = 0; c < r; ++c) {
        for (int i = 0; i < m; ++i) {
            cplx acc = 0.0;
            for (int q = 0; q < ell; ++q) acc += Q(i, q) * d.U(q, c);
            U(i, c) = acc;
        }
        for (int j = 0; j < n; ++j) V(c, j) = d.s[c] * std::conj(d.V(j, c));
    }
    return true;
}

}  // namespace fdbem
