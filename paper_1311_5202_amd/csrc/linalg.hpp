// Small dense complex linear algebra for the FP64 set-up of translation
// operators: column-major matrices, products, a one-sided Jacobi SVD and a
// greedy column skeleton selection (pivoted Gram-Schmidt).  Sizes here are a
// few hundred at most, so plain loops are enough.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace fdbem {

using cplx = std::complex<double>;

struct CMat {
    int m = 0, n = 0;            // rows, cols
    std::vector<cplx> a;         // column-major, a[i + j*m]
    CMat() = default;
    CMat(int rows, int cols) : m(rows), n(cols), a((size_t)rows * cols) {}
    cplx &operator()(int i, int j) { return a[(size_t)i + (size_t)j * m]; }
    const cplx &operator()(int i, int j) const { return a[(size_t)i + (size_t)j * m]; }
    cplx *col(int j) { return a.data() + (size_t)j * m; }
    const cplx *col(int j) const { return a.data() + (size_t)j * m; }
};

// C = op(A) * op(B); op is 'N' (none), 'T' (transpose), 'C' (conjugate transpose)
CMat matmul(const CMat &A, char opA, const CMat &B, char opB);

struct SVD {
    CMat U;                      // m x r
    std::vector<double> s;       // r, descending
    CMat V;                      // n x r   (A ~= U diag(s) V^H)
};

// Thin SVD by one-sided Jacobi on the columns (after a QR if m > n is large).
SVD svd(const CMat &A);

// Number of singular values with s_i >= eps * s_0.
int truncation_rank(const std::vector<double> &s, double eps);

// Greedy column selection: indices of up to max_k columns chosen by
// pivoted Gram-Schmidt, stopping once the largest remaining column norm
// drops below tol * (largest initial norm).
std::vector<int> select_columns(const CMat &A, double tol, int max_k);

// Gaussian sketch rows: returns (k x A.m) matrix with N(0,1)/sqrt(k) entries
// (complex), deterministic in seed.
CMat gaussian_sketch(int k, int m, uint64_t seed);

// Orthonormal columns spanning those of A (Gram-Schmidt twice); a column
// that vanishes is replaced by a coordinate vector orthogonal to the rest.
void orthonormalize(CMat &A);

// Factors A ~= U V (U: m x r, V: r x n) truncated at sigma_i >= eps sigma_1,
// found by a randomized range finder with one power iteration when the
// eps-rank is at most max_r; returns false (and leaves U, V) otherwise.
bool lowrank_factor(const CMat &A, double eps, int max_r, uint64_t seed, CMat &U, CMat &V, int &r);

}  // namespace fdbem
