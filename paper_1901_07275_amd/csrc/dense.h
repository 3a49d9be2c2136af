// Small dense complex linear algebra for the host plan: Householder QR with
// column pivoting, one-sided Jacobi SVD and the pseudo-inverse built on it.
// These are the building blocks Algorithm 2.1 (Section 2.1) asks for
// (pivoted QR / LQ of sampled rows and columns, pseudo-inverses, a small SVD).
// Column-major storage throughout; sizes here are O(rank) x n at most.
#pragma once

#include <complex>
#include <vector>

namespace jt {

using cd = std::complex<double>;

struct CMat {
    int rows = 0, cols = 0;
    std::vector<cd> a;  // column-major
    CMat() = default;
    CMat(int r, int c) : rows(r), cols(c), a((size_t)r * c, cd(0.0, 0.0)) {}
    cd &operator()(int i, int j) { return a[(size_t)i + (size_t)j * rows]; }
    const cd &operator()(int i, int j) const { return a[(size_t)i + (size_t)j * rows]; }
};

CMat adjoint(const CMat &m);
CMat matmul(const CMat &x, const CMat &y);

// Householder QR with column pivoting of m (rows x cols), run for at most
// `steps` steps.  Returns the column order chosen (first entries = pivots).
// If q_out is non-null it receives the first `steps` columns of Q.
std::vector<int> pivoted_qr(const CMat &m, int steps, CMat *q_out);

// Thin SVD  m = U diag(s) V^*  of an m x k matrix (any shape) by one-sided
// Jacobi on the taller orientation.  Singular values are sorted descending.
void svd(const CMat &m, CMat &U, std::vector<double> &s, CMat &V);

// Moore-Penrose pseudo-inverse; singular values below rcond * s_max are dropped.
CMat pinv(const CMat &m, double rcond = 1e-14);

}  // namespace jt
