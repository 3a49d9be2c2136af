/*
 * Reference (oracle) construction of the uniform Jacobi transform matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU baseline
 * of the benchmark use it.  It shares no code with the GPU path or the host
 * plan: every routine below is written out again here on purpose.
 *
 * What it computes (Section 3.1, eqs. (35)-(39), with the orthonormalisation
 * of eq. (7) and the quadrature of eqs. (2) and (9)):
 *
 *     A[j][k] = sqrt(omega_j) * phat_k(x_j),   j, k = 0 .. n-1
 *
 * where x_j are the n Gauss-Jacobi nodes for the weight
 * w(x) = (1-x)^a (1+x)^b on [-1,1] (eq. (2); the printed weight
 * "(1+x)^a (1+x)^b" is read as (1-x)^a (1+x)^b), ordered by ascending
 * t_j = arccos(x_j) (descending x), omega_j the Gauss-Jacobi weights, and
 * phat_k = P_k^(a,b) / ||P_k^(a,b)|| the orthonormal Jacobi polynomials.
 * Substituting eq. (5) and the change of variables x = cos t behind eq. (9)
 * into sqrt(w_j) Ptilde_k(t_j) gives exactly this expression, so A is the
 * matrix W J_n^(a,b) of Section 3.1, which the paper states is orthogonal.
 *
 * Steps (all internal arithmetic in long double, 64-bit mantissa on x86):
 *   O1  recurrence coefficients of the orthonormal family (textbook Jacobi
 *       three-term recurrence; the paper only says "three-term recurrence"),
 *       with the a+b = 0 and a+b = -1 special cases written out;
 *   O2  nodes = eigenvalues of the symmetric tridiagonal Jacobi matrix
 *       (Golub-Welsch), found one by one by Sturm-sequence bisection;
 *   O3  two Newton steps on phat_n at each node;
 *   O4  order by descending x (ascending t);
 *   O5  phat_k(x_j) for k < n by the recurrence, and the Christoffel weights
 *       omega_j = 1 / sum_{k<n} phat_k(x_j)^2;
 *   O6  A[j][k] = sqrt(omega_j) phat_k(x_j), rounded to double.
 * Parity pins for every step live in tests/test_oracle_pins.py.
 *
 * Two further entry points at the end of this file:
 *   orc_ptilde       the modified Jacobi functions Ptilde_k(t) at arbitrary
 *                    angles (the nonuniform forward transform);
 *   orc_nodes_fp64,  the same uniform 1D definition in plain fp64, for long
 *   orc_apply_fp64   items where the long double build is too slow.  Its
 *                    accuracy at the end nodes is about n^2 * 1e-16 (fp64 x
 *                    next to +-1), enough to check fp32-bulk results.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

typedef long double ld;

/* O1: coefficients of  x phat_k = beta_{k+1} phat_{k+1} + alpha_k phat_k + beta_k phat_{k-1}. */
static void orc_coeffs(int n, ld a, ld b, ld *alpha, ld *beta, ld *mu0)
{
    for (int k = 0; k <= n; ++k) {
        if (k == 0) {
            alpha[0] = (b - a) / (a + b + 2.0L);
        } else {
            ld s = 2.0L * k + a + b;
            alpha[k] = (b * b - a * a) / (s * (s + 2.0L));
        }
    }
    beta[0] = 0.0L;
    for (int k = 1; k <= n; ++k) {
        if (k == 1) {
            /* the general formula is 0/0 when a+b = -1; this is its limit form */
            beta[1] = sqrtl(4.0L * (1.0L + a) * (1.0L + b)
                            / ((a + b + 2.0L) * (a + b + 2.0L) * (a + b + 3.0L)));
        } else {
            ld s = 2.0L * k + a + b;
            ld num = 4.0L * k * (k + a) * (k + b) * (k + a + b);
            ld den = s * s * (s + 1.0L) * (s - 1.0L);
            beta[k] = sqrtl(num / den);
        }
    }
    /* mu0 = integral of w over [-1,1] = 2^(a+b+1) Gamma(a+1) Gamma(b+1) / Gamma(a+b+2) */
    *mu0 = expl((a + b + 1.0L) * logl(2.0L) + lgammal(a + 1.0L) + lgammal(b + 1.0L)
                - lgammal(a + b + 2.0L));
}

/* phat_n(x) and its derivative by the recurrence. */
static void orc_eval_pn(int n, const ld *alpha, const ld *beta, ld mu0, ld x, ld *p, ld *dp)
{
    ld pm1 = 0.0L, dpm1 = 0.0L;
    ld pk = 1.0L / sqrtl(mu0), dpk = 0.0L;
    for (int k = 0; k < n; ++k) {
        ld pn = ((x - alpha[k]) * pk - beta[k] * pm1) / beta[k + 1];
        ld dpn = ((x - alpha[k]) * dpk + pk - beta[k] * dpm1) / beta[k + 1];
        pm1 = pk; dpm1 = dpk;
        pk = pn; dpk = dpn;
    }
    *p = pk;
    *dp = dpk;
}

/* Number of eigenvalues of the n x n Jacobi matrix that are < x (Sturm count
 * through the LDL^T pivots of J - xI). */
static int orc_sturm_count(int n, const ld *alpha, const ld *beta, ld x)
{
    int cnt = 0;
    ld q = 1.0L;
    for (int i = 0; i < n; ++i) {
        ld off2 = (i == 0) ? 0.0L : beta[i] * beta[i];
        if (i == 0)
            q = alpha[0] - x;
        else
            q = (alpha[i] - x) - off2 / q;
        if (q == 0.0L)
            q = -1e-4000L; /* perturb an exact zero pivot to the negative side */
        if (q < 0.0L)
            ++cnt;
    }
    return cnt;
}

/*
 * Build A (n x n, row-major A[j*n+k]), nodes x (descending) and weights omega.
 * Any output pointer may be NULL.  Returns 0 on success, nonzero on bad input.
 */
int orc_build(int n, double a_in, double b_in, double *A, double *x_out, double *w_out)
{
    if (n < 1 || !(a_in > -1.0) || !(b_in > -1.0))
        return 1;
    ld a = a_in, b = b_in;
    ld *alpha = (ld *)malloc(sizeof(ld) * (n + 1));
    ld *beta = (ld *)malloc(sizeof(ld) * (n + 1));
    ld *x = (ld *)malloc(sizeof(ld) * n);
    ld *om = (ld *)malloc(sizeof(ld) * n);
    if (!alpha || !beta || !x || !om) {
        free(alpha); free(beta); free(x); free(om);
        return 2;
    }
    ld mu0;
    orc_coeffs(n, a, b, alpha, beta, &mu0);

    /* O2 + O3: the i-th smallest eigenvalue by bisection on [-1, 1], then Newton. */
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        ld lo = -1.0L, hi = 1.0L;
        for (int it = 0; it < 80; ++it) {
            ld mid = 0.5L * (lo + hi);
            if (orc_sturm_count(n, alpha, beta, mid) > i)
                hi = mid;
            else
                lo = mid;
            if (hi - lo < 1e-13L)
                break;
        }
        ld xi = 0.5L * (lo + hi);
        for (int it = 0; it < 3; ++it) {
            ld p, dp;
            orc_eval_pn(n, alpha, beta, mu0, xi, &p, &dp);
            if (dp != 0.0L)
                xi -= p / dp;
        }
        /* O4: eigenvalue i (ascending x) goes to slot n-1-i (ascending t) */
        x[n - 1 - i] = xi;
    }

    /* O5 + O6 */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        ld xj = x[j];
        ld pm1 = 0.0L, pk = 1.0L / sqrtl(mu0);
        ld sum = 0.0L;
        ld *row = (ld *)malloc(sizeof(ld) * n);
        for (int k = 0; k < n; ++k) {
            row[k] = pk;
            sum += pk * pk;
            ld pn = ((xj - alpha[k]) * pk - beta[k] * pm1) / beta[k + 1];
            pm1 = pk;
            pk = pn;
        }
        om[j] = 1.0L / sum;
        if (A) {
            ld s = sqrtl(om[j]);
            for (int k = 0; k < n; ++k)
                A[(size_t)j * n + k] = (double)(s * row[k]);
        }
        free(row);
    }
    if (x_out)
        for (int j = 0; j < n; ++j) x_out[j] = (double)x[j];
    if (w_out)
        for (int j = 0; j < n; ++j) w_out[j] = (double)om[j];
    free(alpha); free(beta); free(x); free(om);
    return 0;
}

/* Recurrence coefficients alone (for the pins that check O1 by itself). */
int orc_recurrence(int n, double a_in, double b_in, double *alpha_out, double *beta_out, double *mu0_out)
{
    if (n < 1 || !(a_in > -1.0) || !(b_in > -1.0))
        return 1;
    ld *alpha = (ld *)malloc(sizeof(ld) * (n + 1));
    ld *beta = (ld *)malloc(sizeof(ld) * (n + 1));
    ld mu0;
    orc_coeffs(n, a_in, b_in, alpha, beta, &mu0);
    for (int k = 0; k <= n; ++k) {
        alpha_out[k] = (double)alpha[k];
        beta_out[k] = (double)beta[k];
    }
    *mu0_out = (double)mu0;
    free(alpha); free(beta);
    return 0;
}

/* ======================================================================
 * Modified Jacobi functions at given angles (the nonuniform transform).
 *
 * Ptilde_k(t) = phat_k(cos t) * sqrt(w(cos t) sin t),  w(x) = (1-x)^a (1+x)^b,
 * which is the normalisation that makes {Ptilde_k} orthonormal on (0, pi)
 * (the modified Jacobi functions of the first kind, Section 1, with the
 * substitution x = cos t).  w(cos t) sin t is formed as
 * 2^(a+b+1) sin(t/2)^(2a+1) cos(t/2)^(2b+1), without cancellation near the ends.
 * The nonuniform forward transform (Section 3.1, the remark after eq. (39))
 * is f_j = sum_{k<n} alpha_k Ptilde_k(t_j) at arbitrary t_j in (0, pi), with
 * no quadrature weights.
 * out: m x n row-major, out[j*n + k] = Ptilde_k(t_j).  Long double inside.
 * ====================================================================== */
int orc_ptilde(int n, double a_in, double b_in, int m, const double *t_in, double *out)
{
    if (n < 1 || m < 0 || !(a_in > -1.0) || !(b_in > -1.0))
        return 1;
    for (int j = 0; j < m; ++j)
        if (!(t_in[j] > 0.0) || !(t_in[j] < 3.14159265358979323846))
            return 3;
    ld a = a_in, b = b_in;
    ld *alpha = (ld *)malloc(sizeof(ld) * (n + 1));
    ld *beta = (ld *)malloc(sizeof(ld) * (n + 1));
    if (!alpha || !beta) {
        free(alpha); free(beta);
        return 2;
    }
    ld mu0;
    orc_coeffs(n, a, b, alpha, beta, &mu0);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < m; ++j) {
        ld t = t_in[j];
        ld x = cosl(t);
        ld sh = sinl(t / 2.0L), ch = cosl(t / 2.0L);
        ld scale = sqrtl(powl(2.0L, a + b + 1.0L) * powl(sh, 2.0L * a + 1.0L) * powl(ch, 2.0L * b + 1.0L));
        ld pm1 = 0.0L, pk = 1.0L / sqrtl(mu0);
        for (int k = 0; k < n; ++k) {
            out[(size_t)j * n + k] = (double)(scale * pk);
            ld pn = ((x - alpha[k]) * pk - beta[k] * pm1) / beta[k + 1];
            pm1 = pk;
            pk = pn;
        }
    }
    free(alpha); free(beta);
    return 0;
}

/* ======================================================================
 * The uniform 1D transform in plain fp64, for sizes where the long double
 * construction above is too slow to check many items (the same definition:
 * A[j][k] = sqrt(omega_j) phat_k(x_j), nodes ascending in t).
 *
 *   nodes   : the n zeros of phat_n.  Each is isolated by a sign change of
 *             phat_n on a uniform grid in t = arccos x (the grid is doubled
 *             until exactly n sign changes are seen: phat_n has n simple
 *             zeros in (-1, 1), so then every interval holds exactly one),
 *             then refined by Newton's method on phat_n, with a bisection
 *             step whenever Newton would leave the interval.
 *   weights : Christoffel, omega_j = 1 / sum_{k<n} phat_k(x_j)^2.
 *   apply   : forward g_j = sqrt(omega_j) sum_k phat_k(x_j) alpha_k;
 *             inverse alpha_k = sum_j sqrt(omega_j) phat_k(x_j) g_j.
 * The recurrence runs over k in the outer loop and over points in the inner
 * loop (independent points side by side).  No matrix is stored.
 * ====================================================================== */
#define ORC_BLK 256

typedef struct {
    int n;
    double *al, *be, *ibe; /* alpha_k, beta_k, 1/beta_k (k <= n) */
    double p0;             /* phat_0 = mu0^(-1/2) */
} orc_rec_d;

static int orc_rec_d_init(orc_rec_d *r, int n, double a, double b)
{
    ld *al = (ld *)malloc(sizeof(ld) * (n + 1));
    ld *be = (ld *)malloc(sizeof(ld) * (n + 1));
    r->n = n;
    r->al = (double *)malloc(sizeof(double) * (n + 1));
    r->be = (double *)malloc(sizeof(double) * (n + 1));
    r->ibe = (double *)malloc(sizeof(double) * (n + 1));
    if (!al || !be || !r->al || !r->be || !r->ibe) {
        free(al); free(be); free(r->al); free(r->be); free(r->ibe);
        return 2;
    }
    ld mu0;
    orc_coeffs(n, a, b, al, be, &mu0);
    for (int k = 0; k <= n; ++k) {
        r->al[k] = (double)al[k];
        r->be[k] = (double)be[k];
        r->ibe[k] = k > 0 ? (double)(1.0L / be[k]) : 0.0;
    }
    r->p0 = (double)(1.0L / sqrtl(mu0));
    free(al); free(be);
    return 0;
}

static void orc_rec_d_free(orc_rec_d *r)
{
    free(r->al); free(r->be); free(r->ibe);
}

/* phat_n (and, if dp != NULL, phat_n') at m <= ORC_BLK points. */
static void orc_pn_d(const orc_rec_d *r, int m, const double *x, double *p, double *dp)
{
    double pm[ORC_BLK], pk[ORC_BLK], dpm[ORC_BLK], dpk[ORC_BLK];
    for (int i = 0; i < m; ++i) {
        pm[i] = 0.0; pk[i] = r->p0; dpm[i] = 0.0; dpk[i] = 0.0;
    }
    for (int k = 0; k < r->n; ++k) {
        const double ak = r->al[k], bk = r->be[k], ib = r->ibe[k + 1];
        if (dp) {
            for (int i = 0; i < m; ++i) {
                double pn = ((x[i] - ak) * pk[i] - bk * pm[i]) * ib;
                double dpn = ((x[i] - ak) * dpk[i] + pk[i] - bk * dpm[i]) * ib;
                pm[i] = pk[i]; pk[i] = pn;
                dpm[i] = dpk[i]; dpk[i] = dpn;
            }
        } else {
            for (int i = 0; i < m; ++i) {
                double pn = ((x[i] - ak) * pk[i] - bk * pm[i]) * ib;
                pm[i] = pk[i]; pk[i] = pn;
            }
        }
    }
    for (int i = 0; i < m; ++i) {
        p[i] = pk[i];
        if (dp) dp[i] = dpk[i];
    }
}

static int orc_sign(double v) { return v < 0.0 ? -1 : 1; }

/* Nodes (descending x = ascending t) and Christoffel weights in fp64.
 * Returns 0, or 4 if the zeros could not be isolated. */
int orc_nodes_fp64(int n, double a, double b, double *x_out, double *w_out)
{
    if (n < 1 || !(a > -1.0) || !(b > -1.0))
        return 1;
    orc_rec_d r;
    if (orc_rec_d_init(&r, n, a, b))
        return 2;
    const double pi = 3.14159265358979323846;
    int rc = 4;
    double *lo = (double *)malloc(sizeof(double) * n);
    double *hi = (double *)malloc(sizeof(double) * n);
    /* consecutive zeros are about pi/n apart in t, so a grid of 2n steps
     * usually isolates all of them; it is refined until it does */
    for (int M = 2 * n + 2; M <= 64 * n + 64 && rc == 4; M *= 2) {
        double *s = (double *)malloc(sizeof(double) * (M + 1));
        /* phat_n on the grid t_i = pi i / M, i = 0..M */
#pragma omp parallel for schedule(dynamic, 1)
        for (int i0 = 0; i0 <= M; i0 += ORC_BLK) {
            double xs[ORC_BLK];
            int m = (M + 1 - i0) < ORC_BLK ? (M + 1 - i0) : ORC_BLK;
            for (int i = 0; i < m; ++i) xs[i] = cos(pi * (double)(i0 + i) / (double)M);
            orc_pn_d(&r, m, xs, s + i0, NULL);
        }
        int cnt = 0;
        /* a zero that falls exactly on a grid point is counted once, with
         * the interval that ends there (the next interval is skipped) */
        for (int i = 0; i < M && cnt <= n; ++i)
            if (s[i] != 0.0 && (s[i + 1] == 0.0 || orc_sign(s[i]) != orc_sign(s[i + 1]))) {
                if (cnt < n) {
                    hi[cnt] = cos(pi * (double)i / (double)M);       /* x decreases with t */
                    lo[cnt] = cos(pi * (double)(i + 1) / (double)M);
                }
                ++cnt;
            }
        free(s);
        if (cnt == n) rc = 0;
    }
    if (rc == 0) {
        /* safeguarded Newton inside each interval, points side by side */
#pragma omp parallel for schedule(dynamic, 1)
        for (int j0 = 0; j0 < n; j0 += ORC_BLK) {
            int m = (n - j0) < ORC_BLK ? (n - j0) : ORC_BLK;
            double xs[ORC_BLK], l[ORC_BLK], h[ORC_BLK], slo[ORC_BLK], p[ORC_BLK], dp[ORC_BLK];
            int active[ORC_BLK];
            for (int i = 0; i < m; ++i) {
                l[i] = lo[j0 + i]; h[i] = hi[j0 + i];
                xs[i] = 0.5 * (l[i] + h[i]);
                active[i] = 1;
            }
            orc_pn_d(&r, m, l, slo, NULL);
            for (int i = 0; i < m; ++i)
                if (slo[i] == 0.0) { /* the zero sits on the grid point itself */
                    xs[i] = l[i];
                    active[i] = 0;
                }
            for (int it = 0; it < 200; ++it) {
                int any = 0;
                orc_pn_d(&r, m, xs, p, dp);
                for (int i = 0; i < m; ++i) {
                    if (!active[i]) continue;
                    if (p[i] == 0.0) { active[i] = 0; continue; }
                    if (orc_sign(p[i]) == orc_sign(slo[i])) l[i] = xs[i]; else h[i] = xs[i];
                    double xn = (dp[i] != 0.0) ? xs[i] - p[i] / dp[i] : 0.5 * (l[i] + h[i]);
                    /* Newton converges quadratically here, so a step of a few
                     * units in the last place leaves a smaller error behind
                     * (tested before the safeguard: at the zero itself the
                     * step may point just past the bracket end it sits on) */
                    if (fabs(xn - xs[i]) <= 8.0 * DBL_EPSILON) {
                        active[i] = 0;
                        continue;
                    }
                    if (!(xn >= l[i] && xn <= h[i])) xn = 0.5 * (l[i] + h[i]);
                    xs[i] = xn;
                    if (h[i] - l[i] <= 8.0 * DBL_EPSILON)
                        active[i] = 0;
                    else
                        any = 1;
                }
                if (!any) break;
            }
            for (int i = 0; i < m; ++i) x_out[j0 + i] = xs[i];
        }
        if (w_out) {
#pragma omp parallel for schedule(dynamic, 1)
            for (int j0 = 0; j0 < n; j0 += ORC_BLK) {
                int m = (n - j0) < ORC_BLK ? (n - j0) : ORC_BLK;
                double pm[ORC_BLK], pk[ORC_BLK], sum[ORC_BLK];
                for (int i = 0; i < m; ++i) { pm[i] = 0.0; pk[i] = r.p0; sum[i] = 0.0; }
                for (int k = 0; k < n; ++k) {
                    const double ak = r.al[k], bk = r.be[k], ib = r.ibe[k + 1];
                    for (int i = 0; i < m; ++i) {
                        sum[i] += pk[i] * pk[i];
                        double pn = ((x_out[j0 + i] - ak) * pk[i] - bk * pm[i]) * ib;
                        pm[i] = pk[i]; pk[i] = pn;
                    }
                }
                for (int i = 0; i < m; ++i) w_out[j0 + i] = 1.0 / sum[i];
            }
        }
    }
    free(lo); free(hi);
    orc_rec_d_free(&r);
    return rc;
}

/* Uniform 1D transform of one vector in fp64: forward (transpose = 0)
 * y = A v, inverse (transpose = 1) y = A^T v, with A built from the nodes of
 * orc_nodes_fp64.  Returns 0 or the node finder's code. */
int orc_apply_fp64(int n, double a, double b, int transpose, const double *v, double *y)
{
    double *x = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    if (!x || !w) { free(x); free(w); return 2; }
    int rc = orc_nodes_fp64(n, a, b, x, w);
    orc_rec_d r;
    if (rc == 0 && orc_rec_d_init(&r, n, a, b)) rc = 2;
    if (rc == 0) {
        if (!transpose) {
#pragma omp parallel for schedule(dynamic, 1)
            for (int j0 = 0; j0 < n; j0 += ORC_BLK) {
                int m = (n - j0) < ORC_BLK ? (n - j0) : ORC_BLK;
                double pm[ORC_BLK], pk[ORC_BLK], acc[ORC_BLK];
                for (int i = 0; i < m; ++i) { pm[i] = 0.0; pk[i] = r.p0; acc[i] = 0.0; }
                for (int k = 0; k < n; ++k) {
                    const double ak = r.al[k], bk = r.be[k], ib = r.ibe[k + 1], vk = v[k];
                    for (int i = 0; i < m; ++i) {
                        acc[i] += pk[i] * vk;
                        double pn = ((x[j0 + i] - ak) * pk[i] - bk * pm[i]) * ib;
                        pm[i] = pk[i]; pk[i] = pn;
                    }
                }
                for (int i = 0; i < m; ++i) y[j0 + i] = sqrt(w[j0 + i]) * acc[i];
            }
        } else {
            int nblk = (n + ORC_BLK - 1) / ORC_BLK;
            double *part = (double *)calloc((size_t)nblk * n, sizeof(double));
            if (!part) rc = 2;
            if (rc == 0) {
#pragma omp parallel for schedule(dynamic, 1)
                for (int bi = 0; bi < nblk; ++bi) {
                    int j0 = bi * ORC_BLK;
                    int m = (n - j0) < ORC_BLK ? (n - j0) : ORC_BLK;
                    double pm[ORC_BLK], pk[ORC_BLK], c[ORC_BLK];
                    for (int i = 0; i < m; ++i) { pm[i] = 0.0; pk[i] = r.p0; c[i] = sqrt(w[j0 + i]) * v[j0 + i]; }
                    double *pa = part + (size_t)bi * n;
                    for (int k = 0; k < n; ++k) {
                        const double ak = r.al[k], bk = r.be[k], ib = r.ibe[k + 1];
                        double s = 0.0;
                        for (int i = 0; i < m; ++i) {
                            s += c[i] * pk[i];
                            double pn = ((x[j0 + i] - ak) * pk[i] - bk * pm[i]) * ib;
                            pm[i] = pk[i]; pk[i] = pn;
                        }
                        pa[k] = s;
                    }
                }
                for (int k = 0; k < n; ++k) {
                    double s = 0.0;
                    for (int bi = 0; bi < nblk; ++bi) s += part[(size_t)bi * n + k];
                    y[k] = s;
                }
            }
            free(part);
        }
        orc_rec_d_free(&r);
    }
    free(x); free(w);
    return rc;
}

/* ======================================================================
 * Modified Jacobi functions of the second kind (Section 1: Qtilde_k, the
 * companion of Ptilde_k in Ptilde_k + i Qtilde_k = M exp(i psi)).
 *
 * The paper defines Qtilde_k through the Jacobi function of the second kind
 * and leaves its normalisation to the literature.  The reading used here
 * (the one under which Ptilde_k + i Qtilde_k has a non-oscillatory amplitude
 * and an increasing phase, and which reduces to the sine/cosine pairs of the
 * Chebyshev cases) is
 *
 *     Qtilde_k(t) = sqrt(sin t / w(x)) q_k(x) / pi,   x = cos t,
 *     q_k(x)      = PV int_{-1}^{1} w(s) phat_k(s) / (s - x) ds,
 *
 * i.e. the finite Hilbert transform of w phat_k.  From
 * s phat_k = beta_{k+1} phat_{k+1} + alpha_k phat_k + beta_k phat_{k-1}:
 *     beta_{k+1} q_{k+1} = (x - alpha_k) q_k - beta_k q_{k-1} + [k = 0] sqrt(mu0),
 * and q_0 = H(x) / sqrt(mu0) with H(x) = PV int w(s) / (s - x) ds, written in
 * closed form (Tricomi) for x >= 0:
 *     H(x) = pi cot(pi a) w(x) - 2^(a+b) B(a, b+1) 2F1(1, -a-b; 1-a; (1-x)/2),
 * whose series converges geometrically there ((1-x)/2 <= 1/2); for x < 0 the
 * reflection H^(a,b)(x) = -H^(b,a)(-x) (substitute s -> -s).  For a = b = 0,
 * H(x) = log((1-x)/(1+x)).  The closed form needs a and b away from 0 (the
 * cotangent and Beta function have poles there); those parameters, other
 * than a = b = 0, are refused (code 5).
 * ====================================================================== */
static ld orc_hilbert_pos(ld a, ld b, ld x)
{
    /* x >= 0, a, b not 0 */
    const ld pi = 3.141592653589793238462643383279502884L;
    ld z = (1.0L - x) / 2.0L;
    ld term = 1.0L, sum = 1.0L;
    for (int m = 0; m < 400; ++m) {
        term *= ((ld)m - a - b) / ((ld)m + 1.0L - a) * z;
        sum += term;
        if (fabsl(term) <= 1e-22L * fabsl(sum)) break;
    }
    ld omx = 1.0L - x, opx = 1.0L + x;
    ld w = powl(omx, a) * powl(opx, b);
    /* B(a, b+1) = Gamma(a) Gamma(b+1) / Gamma(a+b+1), with signs (Gamma(a) < 0 for a in (-1, 0)) */
    ld beta_ab = tgammal(a) * tgammal(b + 1.0L) / tgammal(a + b + 1.0L);
    ld cot = cosl(pi * a) / sinl(pi * a);
    return pi * cot * w - powl(2.0L, a + b) * beta_ab * sum;
}

static int orc_hilbert(ld a, ld b, ld x, ld *h)
{
    if (a == 0.0L && b == 0.0L) {
        *h = logl((1.0L - x) / (1.0L + x));
        return 0;
    }
    if (a == 0.0L || b == 0.0L)
        return 5;
    *h = (x >= 0.0L) ? orc_hilbert_pos(a, b, x) : -orc_hilbert_pos(b, a, -x);
    return 0;
}

/* out: m x n row-major, out[j*n + k] = Qtilde_k(t_j) at t_j in (0, pi). */
int orc_qtilde(int n, double a_in, double b_in, int m, const double *t_in, double *out)
{
    if (n < 1 || m < 0 || !(a_in > -1.0) || !(b_in > -1.0) || !(a_in < 1.0) || !(b_in < 1.0))
        return 1;
    if ((a_in == 0.0) != (b_in == 0.0))
        return 5;
    for (int j = 0; j < m; ++j)
        if (!(t_in[j] > 0.0) || !(t_in[j] < 3.14159265358979323846))
            return 3;
    ld a = a_in, b = b_in;
    ld *alpha = (ld *)malloc(sizeof(ld) * (n + 1));
    ld *beta = (ld *)malloc(sizeof(ld) * (n + 1));
    if (!alpha || !beta) {
        free(alpha); free(beta);
        return 2;
    }
    ld mu0;
    orc_coeffs(n, a, b, alpha, beta, &mu0);
    const ld pi = 3.141592653589793238462643383279502884L;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int j = 0; j < m; ++j) {
        ld t = t_in[j];
        ld sh = sinl(t / 2.0L), ch = cosl(t / 2.0L);
        ld omx = 2.0L * sh * sh, opx = 2.0L * ch * ch; /* 1 - x, 1 + x */
        ld x = cosl(t);
        ld w = powl(omx, a) * powl(opx, b);
        ld h;
        if (orc_hilbert(a, b, x, &h)) { bad = 1; continue; }
        ld scale = sqrtl(sinl(t) / w) / pi;
        ld qm1 = 0.0L, qk = h / sqrtl(mu0);
        for (int k = 0; k < n; ++k) {
            out[(size_t)j * n + k] = (double)(scale * qk);
            ld qn = ((x - alpha[k]) * qk - beta[k] * qm1 + (k == 0 ? sqrtl(mu0) : 0.0L)) / beta[k + 1];
            qm1 = qk;
            qk = qn;
        }
    }
    free(alpha); free(beta);
    return bad ? 5 : 0;
}

/* Uniform second-kind matrix at the Gauss-Jacobi nodes, the weighted
 * counterpart of orc_build: Q[j][k] = sqrt(w_j) Qtilde_k(t_j) with the
 * trigonometric weights w_j = omega_j / (w(x_j) sin t_j) of eq. (9), i.e.
 * sqrt(omega_j) q_k(x_j) / (pi w(x_j)).  The nodes and weights are those of
 * orc_build (same steps O1-O5), recomputed here in long double. */
int orc_build_q(int n, double a_in, double b_in, double *Q)
{
    if (n < 1 || !(a_in > -1.0) || !(b_in > -1.0) || !(a_in < 1.0) || !(b_in < 1.0))
        return 1;
    if ((a_in == 0.0) != (b_in == 0.0))
        return 5;
    ld a = a_in, b = b_in;
    ld *alpha = (ld *)malloc(sizeof(ld) * (n + 1));
    ld *beta = (ld *)malloc(sizeof(ld) * (n + 1));
    ld *x = (ld *)malloc(sizeof(ld) * n);
    if (!alpha || !beta || !x) {
        free(alpha); free(beta); free(x);
        return 2;
    }
    ld mu0;
    orc_coeffs(n, a, b, alpha, beta, &mu0);
    /* nodes: bisection on the Sturm count, then Newton (as in orc_build) */
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        ld lo = -1.0L, hi = 1.0L;
        for (int it = 0; it < 80; ++it) {
            ld mid = 0.5L * (lo + hi);
            if (orc_sturm_count(n, alpha, beta, mid) > i)
                hi = mid;
            else
                lo = mid;
            if (hi - lo < 1e-13L)
                break;
        }
        ld xi = 0.5L * (lo + hi);
        for (int it = 0; it < 3; ++it) {
            ld p, dp;
            orc_eval_pn(n, alpha, beta, mu0, xi, &p, &dp);
            if (dp != 0.0L)
                xi -= p / dp;
        }
        x[n - 1 - i] = xi;
    }
    const ld pi = 3.141592653589793238462643383279502884L;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int j = 0; j < n; ++j) {
        ld xj = x[j];
        /* Christoffel weight */
        ld pm1 = 0.0L, pk = 1.0L / sqrtl(mu0), sum = 0.0L;
        for (int k = 0; k < n; ++k) {
            sum += pk * pk;
            ld pn = ((xj - alpha[k]) * pk - beta[k] * pm1) / beta[k + 1];
            pm1 = pk;
            pk = pn;
        }
        ld om = 1.0L / sum;
        ld w = powl(1.0L - xj, a) * powl(1.0L + xj, b);
        ld h;
        if (orc_hilbert(a, b, xj, &h)) { bad = 1; continue; }
        ld scale = sqrtl(om) / (pi * w);
        ld qm1 = 0.0L, qk = h / sqrtl(mu0);
        for (int k = 0; k < n; ++k) {
            Q[(size_t)j * n + k] = (double)(scale * qk);
            ld qn = ((xj - alpha[k]) * qk - beta[k] * qm1 + (k == 0 ? sqrtl(mu0) : 0.0L)) / beta[k + 1];
            qm1 = qk;
            qk = qn;
        }
    }
    free(alpha); free(beta); free(x);
    return bad ? 5 : 0;
}
