// Phase and amplitude tables by the third-order ODE for N = M^2 (Section 2.2).
#include "phase.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace jt {

typedef long double ld;
static const ld kPiL = 3.141592653589793238462643383279502884L;

namespace {

constexpr int M = PhaseGrid::kPts;

// Spectral operators on the M Chebyshev-Lobatto points x_i = -cos(pi i/(M-1))
// of [-1, 1] (ascending), all acting on point values:
//   I1 = indefinite integral from -1, I2 = I1^2, I3 = I1^3;
//   d1l/d1r, d2l/d2r = first and second derivative at x = -1 / x = +1;
//   w = barycentric weights of the Lobatto points (eq. (cheby:bary)).
struct Spectral {
    double x[M], w[M];
    double I1[M][M], I2[M][M], I3[M][M];
    double d1l[M], d1r[M], d2l[M], d2r[M];

    Spectral()
    {
        ld xl[M];
        for (int i = 0; i < M; ++i) {
            xl[i] = -cosl(kPiL * i / (M - 1));
            x[i] = (double)xl[i];
            w[i] = (i % 2 ? -1.0 : 1.0) * ((i == 0 || i == M - 1) ? 0.5 : 1.0);
        }
        x[0] = -1.0;
        x[M - 1] = 1.0;
        // V[i][j] = T_j(x_i); Vinv maps values to Chebyshev coefficients
        ld V[M][M], Vinv[M][M];
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) V[i][j] = cosl(j * acosl(std::max((ld)-1, std::min((ld)1, xl[i]))));
        invert(V, Vinv);
        // antiderivative of T_j, zero at -1, evaluated at the points
        auto T = [](int j, ld t) { return cosl(j * acosl(std::max((ld)-1, std::min((ld)1, t)))); };
        auto F = [&](int j, ld t) -> ld {
            if (j == 0) return t;
            if (j == 1) return t * t / 2;
            return (T(j + 1, t) / (j + 1) - T(j - 1, t) / (j - 1)) / 2;
        };
        ld Ib[M][M], A1[M][M], A2[M][M], A3[M][M];
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) Ib[i][j] = F(j, xl[i]) - F(j, (ld)-1);
        mul(Ib, Vinv, A1);
        mul(A1, A1, A2);
        mul(A2, A1, A3);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                I1[i][j] = (double)A1[i][j];
                I2[i][j] = (double)A2[i][j];
                I3[i][j] = (double)A3[i][j];
            }
        // T_j'(+-1) = (+-1)^(j+1) j^2,  T_j''(+-1) = (+-1)^j j^2 (j^2 - 1) / 3
        for (int i = 0; i < M; ++i) {
            ld s1l = 0, s1r = 0, s2l = 0, s2r = 0;
            for (int j = 0; j < M; ++j) {
                const ld j2 = (ld)j * j, e1 = j2, e2 = j2 * (j2 - 1) / 3;
                const ld sg = (j % 2) ? -1 : 1;  // (-1)^j
                s1r += e1 * Vinv[j][i];
                s1l += -sg * e1 * Vinv[j][i];
                s2r += e2 * Vinv[j][i];
                s2l += sg * e2 * Vinv[j][i];
            }
            d1l[i] = (double)s1l; d1r[i] = (double)s1r;
            d2l[i] = (double)s2l; d2r[i] = (double)s2r;
        }
    }

    static void mul(const ld (&A)[M][M], const ld (&B)[M][M], ld (&C)[M][M])
    {
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                ld s = 0;
                for (int k = 0; k < M; ++k) s += A[i][k] * B[k][j];
                C[i][j] = s;
            }
    }
    // Gauss-Jordan with partial pivoting (the Vandermonde matrix of the
    // Chebyshev polynomials at the Lobatto points is well conditioned)
    static void invert(const ld (&A)[M][M], ld (&R)[M][M])
    {
        ld a[M][2 * M];
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < 2 * M; ++j) a[i][j] = j < M ? A[i][j] : (j - M == i ? 1 : 0);
        for (int c = 0; c < M; ++c) {
            int p = c;
            for (int r = c + 1; r < M; ++r)
                if (fabsl(a[r][c]) > fabsl(a[p][c])) p = r;
            for (int j = 0; j < 2 * M; ++j) std::swap(a[c][j], a[p][j]);
            const ld piv = a[c][c];
            for (int j = 0; j < 2 * M; ++j) a[c][j] /= piv;
            for (int r = 0; r < M; ++r)
                if (r != c) {
                    const ld f = a[r][c];
                    if (f != 0)
                        for (int j = 0; j < 2 * M; ++j) a[r][j] -= f * a[c][j];
                }
        }
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) R[i][j] = a[i][M + j];
    }
};

const Spectral &spectral()
{
    static const Spectral s;
    return s;
}

// Solve A s = r (M x M, row-major, destroyed) by Gaussian elimination with
// partial pivoting.
void solve_dense(double (&A)[M][M], double (&r)[M])
{
    for (int c = 0; c < M; ++c) {
        int p = c;
        for (int i = c + 1; i < M; ++i)
            if (std::fabs(A[i][c]) > std::fabs(A[p][c])) p = i;
        if (p != c) {
            for (int j = c; j < M; ++j) std::swap(A[c][j], A[p][j]);
            std::swap(r[c], r[p]);
        }
        const double inv = 1.0 / A[c][c];
        for (int i = c + 1; i < M; ++i) {
            const double f = A[i][c] * inv;
            if (f == 0.0) continue;
            for (int j = c + 1; j < M; ++j) A[i][j] -= f * A[c][j];
            r[i] -= f * r[c];
        }
    }
    for (int c = M - 1; c >= 0; --c) {
        double s = r[c];
        for (int j = c + 1; j < M; ++j) s -= A[c][j] * r[j];
        r[c] = s / A[c][c];
    }
}

// q of eq. (jacobieq:coef) and its t-derivative
struct Coef {
    double lam2, ca, cb;  // lam^2, (1/4 - a^2)/4, (1/4 - b^2)/4
    void at(double t, double &q, double &dq) const
    {
        const double s = std::sin(0.5 * t), c = std::cos(0.5 * t);
        const double s2 = s * s, c2 = c * c;
        q = lam2 + ca / s2 + cb / c2;
        dq = -ca * c / (s2 * s) + cb * s / (c2 * c);
    }
};

// One panel of the ODE in a variable s running from the panel end where the
// values are known (s = 0) to the other end (s = 2h).  qs, dqs: q and dq/ds at
// the points ordered by s; c0, c1, c2: N, dN/ds, d2N/ds2 at s = 0.  Writes N at
// the points (s order) and dN/ds, d2N/ds2 at s = 2h.
void panel_ode(const double *qs, const double *dqs, double h, double c0, double c1, double c2, double *N,
               double &e1, double &e2)
{
    const Spectral &S = spectral();
    const double h2 = h * h, h3 = h2 * h;
    double A[M][M], sig[M], s[M];
    for (int i = 0; i < M; ++i) {
        s[i] = (S.x[i] + 1.0) * h;
        for (int j = 0; j < M; ++j) A[i][j] = 4.0 * qs[i] * h2 * S.I2[i][j] + 2.0 * dqs[i] * h3 * S.I3[i][j];
        A[i][i] += 1.0;
        sig[i] = -4.0 * qs[i] * (c1 + c2 * s[i]) - 2.0 * dqs[i] * (c0 + c1 * s[i] + 0.5 * c2 * s[i] * s[i]);
    }
    solve_dense(A, sig);
    for (int i = 0; i < M; ++i) {
        double i3 = 0.0;
        for (int j = 0; j < M; ++j) i3 += S.I3[i][j] * sig[j];
        N[i] = c0 + c1 * s[i] + 0.5 * c2 * s[i] * s[i] + h3 * i3;
    }
    double i1 = 0.0, i2 = 0.0;
    for (int j = 0; j < M; ++j) {
        i1 += S.I1[M - 1][j] * sig[j];
        i2 += S.I2[M - 1][j] * sig[j];
    }
    const double se = 2.0 * h;
    e1 = c1 + c2 * se + h2 * i2;
    e2 = c2 + h * i1;
}

}  // namespace

PhaseGrid::PhaseGrid(int nmax, double a_, double b_) : a(a_), b(b_)
{
    if (nmax < 2) throw std::invalid_argument("phase grid needs nmax >= 2");
    // l: least integer with (pi/2) 2^(1-l) <= 1/nmax; ends (pi/2) 2^(i-l),
    // i = 1..l, then their reflections pi - (.) down to the smallest
    int l = 2;
    while ((double)(kPiL / 2) * std::ldexp(1.0, 1 - l) > 1.0 / nmax) ++l;
    for (int i = 1; i <= l; ++i) ends.push_back((double)(kPiL / 2 * ldexpl(1.0L, i - l)));
    for (int i = l - 1; i >= 1; --i) ends.push_back((double)(kPiL - kPiL / 2 * ldexpl(1.0L, i - l)));
    data = l - 2;
}

double PhaseGrid::point(int p, int i) const
{
    if (i == 0) return ends[p];
    if (i == M - 1) return ends[p + 1];
    const double h = 0.5 * (ends[p + 1] - ends[p]);
    return ends[p] + (spectral().x[i] + 1.0) * h;
}

int PhaseGrid::panel_of(double t) const
{
    if (!(t >= ends.front()) || !(t <= ends.back())) return -1;
    int p = (int)(std::lower_bound(ends.begin(), ends.end(), t) - ends.begin()) - 1;
    return std::max(0, std::min(p, panels() - 1));
}

void solve_phase(const PhaseGrid &g, double nu, const double *P, const double *Q, DegreePhase &out)
{
    const Spectral &S = spectral();
    const int np = g.panels(), D = g.data;
    const ld laml = (ld)nu + ((ld)g.a + (ld)g.b + 1) / 2;
    const double lam = (double)laml;
    Coef co{lam * lam, (0.25 - g.a * g.a) / 4.0, (0.25 - g.b * g.b) / 4.0};
    out.lam = lam;
    out.N.assign((size_t)np * M, 0.0);
    out.th.assign((size_t)np * M, 0.0);
    double *N = out.N.data();

    // data panel: N = P~^2 + Q~^2; its end derivatives start the ODE
    const double hD = 0.5 * (g.ends[D + 1] - g.ends[D]);
    for (int i = 0; i < M; ++i) N[(size_t)D * M + i] = P[i] * P[i] + Q[i] * Q[i];
    double n1l = 0, n1r = 0, n2l = 0, n2r = 0;
    for (int i = 0; i < M; ++i) {
        const double v = N[(size_t)D * M + i];
        n1l += S.d1l[i] * v; n1r += S.d1r[i] * v;
        n2l += S.d2l[i] * v; n2r += S.d2r[i] * v;
    }
    n1l /= hD; n1r /= hD; n2l /= hD * hD; n2r /= hD * hD;

    double qs[M], dqs[M], Ns[M];
    // toward t = pi: s = t - (left end), the panel's own order
    double c0 = N[(size_t)D * M + M - 1], c1 = n1r, c2 = n2r;
    for (int p = D + 1; p < np; ++p) {
        const double h = 0.5 * (g.ends[p + 1] - g.ends[p]);
        for (int i = 0; i < M; ++i) co.at(g.point(p, i), qs[i], dqs[i]);
        double e1, e2;
        panel_ode(qs, dqs, h, c0, c1, c2, &N[(size_t)p * M], e1, e2);
        c0 = N[(size_t)p * M + M - 1]; c1 = e1; c2 = e2;
    }
    // toward t = 0: s = (right end) - t, reversed order; d/ds = -d/dt
    c0 = N[(size_t)D * M]; c1 = -n1l; c2 = n2l;
    for (int p = D - 1; p >= 0; --p) {
        const double h = 0.5 * (g.ends[p + 1] - g.ends[p]);
        for (int i = 0; i < M; ++i) {
            double q, dq;
            co.at(g.point(p, M - 1 - i), q, dq);
            qs[i] = q; dqs[i] = -dq;
        }
        double e1, e2;
        panel_ode(qs, dqs, h, c0, c1, c2, Ns, e1, e2);
        for (int i = 0; i < M; ++i) N[(size_t)p * M + (M - 1 - i)] = Ns[i];
        c0 = Ns[M - 1]; c1 = e1; c2 = e2;
    }

    // phase: theta' = W / N - lam with W = 2 lam / pi; theta(pi/2) from
    // atan2 on the branch of lam t - (2a + 1) pi / 4
    const double W = 2.0 * lam / (double)kPiL;
    const ld ts = (ld)g.ends[D + 1];
    const ld at = atan2l((ld)Q[M - 1], (ld)P[M - 1]);
    const ld guess = laml * ts - (2 * (ld)g.a + 1) * kPiL / 4;
    const ld m = nearbyintl((guess - at) / (2 * kPiL));
    const double th_star = (double)(at + 2 * kPiL * m - laml * ts);
    double *th = out.th.data();
    auto cumulative = [&](int p, double *C) {
        const double h = 0.5 * (g.ends[p + 1] - g.ends[p]);
        double d[M];
        for (int i = 0; i < M; ++i) d[i] = W / N[(size_t)p * M + i] - lam;
        for (int i = 0; i < M; ++i) {
            double s = 0.0;
            for (int j = 0; j < M; ++j) s += S.I1[i][j] * d[j];
            C[i] = h * s;
        }
    };
    double C[M];
    double val = th_star;
    for (int p = D + 1; p < np; ++p) {
        cumulative(p, C);
        for (int i = 0; i < M; ++i) th[(size_t)p * M + i] = val + C[i];
        val = th[(size_t)p * M + M - 1];
    }
    val = th_star;
    for (int p = D; p >= 0; --p) {
        cumulative(p, C);
        for (int i = 0; i < M; ++i) th[(size_t)p * M + i] = val - (C[M - 1] - C[i]);
        val = th[(size_t)p * M];
    }
}

BaryPoint bary_point(const PhaseGrid &g, double t)
{
    const Spectral &S = spectral();
    BaryPoint bp;
    bp.panel = g.panel_of(t);
    if (bp.panel < 0) throw std::invalid_argument("point outside the phase grid");
    const int p = bp.panel;
    const double h = 0.5 * (g.ends[p + 1] - g.ends[p]);
    const double x = (t - g.ends[p]) / h - 1.0;
    double sum = 0.0;
    for (int i = 0; i < M; ++i) {
        const double d = x - S.x[i];
        if (d == 0.0) {
            for (int k = 0; k < M; ++k) bp.c[k] = (k == i) ? 1.0 : 0.0;
            return bp;
        }
        bp.c[i] = S.w[i] / d;
        sum += bp.c[i];
    }
    for (int i = 0; i < M; ++i) bp.c[i] /= sum;
    return bp;
}

}  // namespace jt
