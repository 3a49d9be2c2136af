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
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

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
