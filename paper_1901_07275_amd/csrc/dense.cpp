#include "dense.h"
#include "threads.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace jt {

CMat adjoint(const CMat &m)
{
    CMat t(m.cols, m.rows);
    for (int j = 0; j < m.cols; ++j)
        for (int i = 0; i < m.rows; ++i) t(j, i) = std::conj(m(i, j));
    return t;
}

CMat matmul(const CMat &x, const CMat &y)
{
    CMat z(x.rows, y.cols);
    for (int j = 0; j < y.cols; ++j)
        for (int l = 0; l < x.cols; ++l) {
            cd yl = y(l, j);
            if (yl == cd(0.0, 0.0)) continue;
            const cd *xc = &x.a[(size_t)l * x.rows];
            cd *zc = &z.a[(size_t)j * z.rows];
            for (int i = 0; i < x.rows; ++i) zc[i] += xc[i] * yl;
        }
    return z;
}

// Column j of a column-major complex matrix as interleaved (re, im) doubles.
static inline double *col_ptr(CMat &m, int j) { return reinterpret_cast<double *>(&m.a[(size_t)j * m.rows]); }

// sum over rows [k, nr) of |c_i|^2.  The reductions in this file may be
// reassociated (vectorized partial sums): the order is fixed by the build, so
// results are reproducible run to run.
static double tail_norm2(const double *c, int k, int nr)
{
#pragma clang fp reassociate(on)
    double s = 0.0;
    for (int i = 2 * k; i < 2 * nr; ++i) s += c[i] * c[i];
    return s;
}

std::vector<int> pivoted_qr(const CMat &m_in, int steps, CMat *q_out)
{
    CMat r = m_in;
    const int nr = r.rows, nc = r.cols;
    steps = std::min(steps, std::min(nr, nc));
    std::vector<int> perm(nc);
    std::iota(perm.begin(), perm.end(), 0);
    std::vector<std::vector<cd>> refl;  // Householder vectors (length nr, zero above k)
    std::vector<double> refl_beta;
    // squared norms of the columns' remaining parts, downdated after every
    // step and recomputed where the downdate has cancelled all but 1e-8 of
    // the value last computed in full (orig)
    std::vector<double> cn(nc), orig(nc);
    parallel_for(nc, [&](int j) { cn[j] = orig[j] = tail_norm2(col_ptr(r, j), 0, nr); });

    for (int k = 0; k < steps; ++k) {
        // pick the column of largest remaining norm
        int best = k;
        double bestn = -1.0;
        for (int j = k; j < nc; ++j)
            if (cn[j] > bestn) { bestn = cn[j]; best = j; }
        if (best != k) {
            for (int i = 0; i < nr; ++i) std::swap(r(i, k), r(i, best));
            std::swap(perm[k], perm[best]);
            std::swap(cn[k], cn[best]);
            std::swap(orig[k], orig[best]);
        }
        // reflector that maps r(k:,k) to a multiple of e_k
        double xn = std::sqrt(tail_norm2(col_ptr(r, k), k, nr));
        std::vector<cd> v(nr, cd(0.0, 0.0));
        if (xn == 0.0) {
            refl.push_back(v);
            refl_beta.push_back(0.0);
            continue;
        }
        cd x0 = r(k, k);
        cd ph = (std::abs(x0) > 0.0) ? x0 / std::abs(x0) : cd(1.0, 0.0);
        for (int i = k; i < nr; ++i) v[i] = r(i, k);
        v[k] += ph * xn;
        double vv = 0.0;
        for (int i = k; i < nr; ++i) vv += std::norm(v[i]);
        double beta = (vv > 0.0) ? 2.0 / vv : 0.0;
        const double *vd = reinterpret_cast<const double *>(v.data());
        parallel_for(nc - k, [&](int jj) {
            const int j = k + jj;
            double *c = col_ptr(r, j);
            // dot = v^H c over rows [k, nr)
            double dr0 = 0.0, di0 = 0.0;
            {
#pragma clang fp reassociate(on)
                for (int i = k; i < nr; ++i) {
                    dr0 += vd[2 * i] * c[2 * i] + vd[2 * i + 1] * c[2 * i + 1];
                    di0 += vd[2 * i] * c[2 * i + 1] - vd[2 * i + 1] * c[2 * i];
                }
            }
            const double dr = beta * dr0, di = beta * di0;
            for (int i2 = k; i2 < nr; ++i2) {
                const double a = vd[2 * i2], b = vd[2 * i2 + 1];
                c[2 * i2] -= a * dr - b * di;
                c[2 * i2 + 1] -= a * di + b * dr;
            }
            if (j > k) {
                const double e = c[2 * k] * c[2 * k] + c[2 * k + 1] * c[2 * k + 1];
                double left = cn[j] - e;
                if (!(left > 1e-8 * orig[j])) orig[j] = left = tail_norm2(c, k + 1, nr);
                cn[j] = left;
            }
        });
        refl.push_back(v);
        refl_beta.push_back(beta);
    }
    if (q_out) {
        CMat q(nr, steps);
        for (int j = 0; j < steps; ++j) q(j, j) = cd(1.0, 0.0);
        for (int k = steps - 1; k >= 0; --k) {
            const std::vector<cd> &v = refl[k];
            double beta = refl_beta[k];
            if (beta == 0.0) continue;
            for (int j = 0; j < steps; ++j) {
                cd dot(0.0, 0.0);
                for (int i = k; i < nr; ++i) dot += std::conj(v[i]) * q(i, j);
                dot *= beta;
                for (int i = k; i < nr; ++i) q(i, j) -= v[i] * dot;
            }
        }
        *q_out = q;
    }
    return perm;
}

// One-sided Jacobi on a tall matrix a (m >= k): a V = U diag(s).
static void jacobi_tall(CMat a, CMat &U, std::vector<double> &s, CMat &V)
{
    const int m = a.rows, k = a.cols;
    V = CMat(k, k);
    for (int i = 0; i < k; ++i) V(i, i) = cd(1.0, 0.0);
    for (int sweep = 0; sweep < 80; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                double al = 0.0, be = 0.0;
                cd ga(0.0, 0.0);
                for (int i = 0; i < m; ++i) {
                    al += std::norm(a(i, p));
                    be += std::norm(a(i, q));
                    ga += std::conj(a(i, p)) * a(i, q);
                }
                double g = std::abs(ga);
                if (g == 0.0 || g <= 1e-15 * std::sqrt(al * be)) continue;
                rotated = true;
                cd ph = ga / g;  // e^{i phi}
                double zeta = (be - al) / (2.0 * g);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
                double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
                // columns: p' = c p - s e^{-i phi} q,  q' = s e^{i phi} p + c q
                for (int i = 0; i < m; ++i) {
                    cd ap = a(i, p), aq = a(i, q);
                    a(i, p) = c * ap - sn * std::conj(ph) * aq;
                    a(i, q) = sn * ph * ap + c * aq;
                }
                for (int i = 0; i < k; ++i) {
                    cd vp = V(i, p), vq = V(i, q);
                    V(i, p) = c * vp - sn * std::conj(ph) * vq;
                    V(i, q) = sn * ph * vp + c * vq;
                }
            }
        if (!rotated) break;
    }
    std::vector<double> nrm(k);
    for (int j = 0; j < k; ++j) {
        double sq = 0.0;
        for (int i = 0; i < m; ++i) sq += std::norm(a(i, j));
        nrm[j] = std::sqrt(sq);
    }
    std::vector<int> ord(k);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
    U = CMat(m, k);
    CMat Vs(k, k);
    s.assign(k, 0.0);
    for (int jj = 0; jj < k; ++jj) {
        int j = ord[jj];
        s[jj] = nrm[j];
        for (int i = 0; i < m; ++i) U(i, jj) = (nrm[j] > 0.0) ? a(i, j) / nrm[j] : cd(0.0, 0.0);
        for (int i = 0; i < k; ++i) Vs(i, jj) = V(i, j);
    }
    V = Vs;
}

void svd(const CMat &m, CMat &U, std::vector<double> &s, CMat &V)
{
    if (m.rows >= m.cols) {
        jacobi_tall(m, U, s, V);
    } else {
        // m^* = V' S U'^*  =>  m = U' S V'^*
        CMat U2, V2;
        jacobi_tall(adjoint(m), U2, s, V2);
        U = V2;
        V = U2;
    }
}

CMat pinv(const CMat &m, double rcond)
{
    CMat U, V;
    std::vector<double> s;
    svd(m, U, s, V);
    const int k = (int)s.size();
    double smax = k ? s[0] : 0.0;
    CMat p(m.cols, m.rows);
    for (int l = 0; l < k; ++l) {
        if (!(s[l] > rcond * smax)) continue;
        double inv = 1.0 / s[l];
        for (int j = 0; j < m.rows; ++j) {
            cd uj = std::conj(U(j, l)) * inv;
            for (int i = 0; i < m.cols; ++i) p(i, j) += V(i, l) * uj;
        }
    }
    return p;
}

}  // namespace jt
