// Host-side plan for the fast uniform Jacobi transform (one axis at a time).
//
// For an axis with n points and parameters (a, b) the plan holds everything
// the device needs to apply W J_n^(a,b) (Section 3.1):
//   * Gauss-Jacobi nodes t_j (ascending) and weights (eq. (2), eq. (9));
//   * DFT bins m_j = [t_j L / 2 pi] (eqs. (45), (47)), L = 2^p >= n;
//   * the direct block W V_n (degrees < nu0, Section 3.1);
//   * the rank-r factors of W B_n from Algorithm 2.1 (Section 2.1, eq. (49)):
//       W B ~ sum_l u_l v_l^T,  u_l = (W U S^1/2)_l,  v_l = (S^1/2 V)_l.
// All of it is computed in long double / double on the host; the device only
// ever sees the packed factor blob.
#pragma once

#include <complex>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace jt {

using cd = std::complex<double>;

struct AxisPlan {
    int n = 0;
    int L = 0;       // FFT length (power of two, >= n, >= 64)
    int nu0 = 0;     // width of the direct block (27, or n for the dense path)
    int rank = 0;    // r
    int max_per_bin = 0;
    bool points = false;  // nonuniform: given points, no quadrature weights (forward only)
    int kind = 1;         // 1: Ptilde (first kind), 2: Qtilde (second kind, forward only)
    int planner = 1;      // 1: recurrence throughout; 2: phase functions for nodes, weights, sampled columns
    double a = 0.0, b = 0.0, tol = 0.0;
    uint64_t seed = 0;
    std::vector<double> t, x, omega;  // nodes ascending in t, Gauss-Jacobi weights (0 for given points)
    std::vector<int32_t> bins;        // m_j in [0, L/2]
    std::vector<int32_t> binptr;      // nodes of bin m: [binptr[m], binptr[m+1]), m <= L/2
    std::vector<double> WV;           // nu0 x n, WV[k*n + j] = sqrt(omega_j) phat_k(x_j)
    std::vector<cd> U;                // rank x n, U[l*n + j]  (weights folded in)
    std::vector<cd> V;                // rank x L, V[l*L + k], zero outside [nu0, n)
    double fro = 0.0;                 // ||W B||_F
    double rel_err = 0.0;             // measured ||W B - U V^T||_F / ||W B||_F
    int rsvd_rounds = 0;
    // offsets of this axis' sections inside the device blob (bytes)
    size_t off_tw64 = 0, off_tw32 = 0, off_bins = 0, off_binptr = 0;
    size_t off_wv64 = 0, off_wv32 = 0, off_u64 = 0, off_u32 = 0, off_v64 = 0, off_v32 = 0;
    size_t bytes = 0;
};

// Widest direct block an FFT-path axis may have: the axis pass keeps the
// inverse direct block's per-degree sums at the front of a line buffer.
constexpr int kMaxNu0 = 64;

struct PlanOptions {
    int nu0 = 27;           // Section 3.1 uses 27; at most kMaxNu0
    int dense_below = 64;   // n < dense_below: the direct block covers all degrees
    int oversample = 2;     // q in Algorithm 2.1
    int iterations = 2;     // repetitions of steps 2-3 (Section 2.1 uses two)
    uint64_t seed = 0;      // 0: derive from (n, a, b, tol)
    int kind = 1;           // 1: first kind, 2: second kind
    int planner = 0;        // 0: automatic, 1: recurrence only, 2: phase functions wherever allowed
};

// Build one axis.  Throws std::runtime_error on bad input or non-convergence.
void build_axis(AxisPlan &ax, int n, double a, double b, double tol, const PlanOptions &opt);

// Build one axis of the nonuniform forward transform at the given points
// t[0..n-1] (non-decreasing, in (0, pi)): rows Ptilde_k(t_j), no weights.
void build_axis_points(AxisPlan &ax, int n, const double *t, double a, double b, double tol,
                       const PlanOptions &opt);

// Exact entries of W B (the low-rank matrix with weights folded in) at
// (row j, degree k) pairs, k in [nu0, n).  For diagnostics and tests.
void exact_entries(const AxisPlan &ax, int count, const int *rows, const int *degs, cd *out);

// Device image of one axis.  layout_axis places the sections at 256-byte
// aligned offsets from `base` (returns the end); precs selects the fp64 and/or
// fp32 copies of the factors (absent sections get offset kAbsent).  pack_axis
// writes the sections into the image starting at dst (offsets count from dst).
constexpr int kPackF64 = 1, kPackF32 = 2;
constexpr size_t kAbsent = ~(size_t)0;
size_t layout_axis(AxisPlan &ax, size_t base, int precs = kPackF64 | kPackF32);
void pack_axis(const AxisPlan &ax, unsigned char *dst);

// Gauss-Jacobi nodes/weights on their own (ascending t), as used by the plan.
void gauss_jacobi(int n, double a, double b, std::vector<double> &t, std::vector<double> &x,
                  std::vector<double> &omega);

// Principal-value integral H(x) = PV int_{-1}^{1} (1-s)^a (1+s)^b / (s - x) ds.
long double hilbert_weight(long double x, long double a, long double b);

}  // namespace jt
