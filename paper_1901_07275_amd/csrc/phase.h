// Nonoscillatory amplitude and phase functions of the modified Jacobi
// functions (Section 2.2): for a degree nu > 27 the pair
//   Ptilde_nu(t) = M(t) cos psi(t),   Qtilde_nu(t) = M(t) sin psi(t)
// has an amplitude whose square N = M^2 solves the third-order linear ODE
// (phase:Neq)
//   N''' + 4 q N' + 2 q' N = 0,
//   q(t) = lam^2 + (1/4 - a^2) / (4 sin^2(t/2)) + (1/4 - b^2) / (4 cos^2(t/2)),
// lam = nu + (a + b + 1)/2 (eq. (jacobieq:coef)), and a phase with
// psi' = W / N, W the pair's Wronskian.
//
// The tables live on the paper's piecewise Chebyshev grid in t: dyadic panels
// (pi/2) 2^(i - m/2) toward t = 0 and their mirror images toward t = pi, the
// smallest reaching below 1 / nmax (eqs. (precomp:tnodes), (precomp:tints)),
// with kPts Chebyshev-Lobatto points on each panel (shared ends).  For one
// degree:
//   * N on the data panel [pi/4, pi/2] is P~^2 + Q~^2 from the three-term
//     recurrence (the caller supplies P~ and Q~ there); its value and first
//     two derivatives at the panel's ends start the ODE, which is solved panel
//     by panel outward toward both ends by spectral collocation of the
//     integral form (the unknown is N''' on the panel's points; N'', N', N
//     are its repeated spectral integrals plus the carried end values; one
//     kPts x kPts solve per panel).  The oscillatory solutions of the ODE are
//     not resolved by the panel grid, so the discrete solve follows the
//     nonoscillatory one (the stiff regime the paper names);
//   * the phase is integrated spectrally from psi(pi/2) = atan2(Q~, P~) with
//     the branch of the large-degree asymptotic lam t - (2a + 1) pi / 4, and
//     stored as theta = psi - lam t (a slowly varying function of size O(1),
//     so the table keeps full double precision).  The Wronskian of the
//     normalized pair is W = 2 lam / pi.
// Values anywhere on the grid then follow by barycentric Chebyshev
// interpolation (eq. (cheby:bary)) on the panel holding t.
#pragma once

#include <cstddef>
#include <vector>

namespace jt {

struct PhaseGrid {
    static constexpr int kPts = 16;   // Chebyshev-Lobatto points per panel
    std::vector<double> ends;         // panel boundaries, ascending (npanels + 1)
    int data = 0;                     // index of the data panel [pi/4, pi/2]
    double a = 0.0, b = 0.0;

    PhaseGrid(int nmax, double a, double b);
    int panels() const { return (int)ends.size() - 1; }
    // point i of panel p (ascending in t)
    double point(int p, int i) const;
    // panel holding t (boundaries go to the lower panel), or -1 outside [ends.front(), ends.back()]
    int panel_of(double t) const;
};

// N and theta = psi - lam t of one degree at every grid point (panel-major,
// kPts values per panel; panel ends appear in both neighbouring panels).
struct DegreePhase {
    double lam = 0.0;
    std::vector<double> N, th;
};

// Solve for degree nu >= 1.  P and Q are Ptilde_nu and Qtilde_nu at the data
// panel's kPts points (ascending in t).
void solve_phase(const PhaseGrid &g, double nu, const double *P, const double *Q, DegreePhase &out);

// Normalized barycentric coefficients of t on its panel: f(t) = sum_i c[i] f_i.
struct BaryPoint {
    int panel = -1;
    double c[PhaseGrid::kPts];
};
BaryPoint bary_point(const PhaseGrid &g, double t);

// N(t) and theta(t) of one degree.
inline void eval_phase(const DegreePhase &d, const BaryPoint &bp, double &N, double &th)
{
    const double *n = &d.N[(size_t)bp.panel * PhaseGrid::kPts], *h = &d.th[(size_t)bp.panel * PhaseGrid::kPts];
    double sn = 0.0, st = 0.0;
    for (int i = 0; i < PhaseGrid::kPts; ++i) {
        sn += bp.c[i] * n[i];
        st += bp.c[i] * h[i];
    }
    N = sn;
    th = st;
}

}  // namespace jt
