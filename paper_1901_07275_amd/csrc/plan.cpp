// Host plan: nodes, weights, bins, direct block, companion function and the
// randomized low-rank factorization of W B_n (Section 2.1, Section 3.1).
#include "plan.h"
#include "threads.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <stdexcept>
#include <thread>

#include "dense.h"
#include "phase.h"

namespace jt {

typedef long double ld;
static const ld kPi = 3.141592653589793238462643383279502884L;


// ------------------------------------------------------------------ RNG
// splitmix64: counter-based, so plans are reproducible for a given key.
struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed) {}
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int below(int m) { return (int)(next() % (uint64_t)m); }
};

static uint64_t mix_key(int n, double a, double b, double tol)
{
    uint64_t h = 0x243F6A8885A308D3ull ^ (uint64_t)n;
    double v[3] = {a, b, tol};
    for (double d : v) {
        uint64_t u;
        std::memcpy(&u, &d, 8);
        Rng r(h ^ u);
        h = r.next();
    }
    return h ? h : 1;
}

// k distinct indices from [0, m) that are not in `excl`, sorted.
static std::vector<int> sample(Rng &rng, int m, int k, const std::vector<int> &excl)
{
    std::vector<char> taken(m, 0);
    for (int e : excl) taken[e] = 1;
    std::vector<int> pool;
    pool.reserve(m);
    for (int i = 0; i < m; ++i)
        if (!taken[i]) pool.push_back(i);
    k = std::min<int>(k, (int)pool.size());
    for (int i = 0; i < k; ++i) {
        int j = i + rng.below((int)pool.size() - i);
        std::swap(pool[i], pool[j]);
    }
    std::vector<int> out(pool.begin(), pool.begin() + k);
    std::sort(out.begin(), out.end());
    return out;
}

static std::vector<int> merged(const std::vector<int> &x, const std::vector<int> &y)
{
    std::vector<int> z(x);
    z.insert(z.end(), y.begin(), y.end());
    std::sort(z.begin(), z.end());
    z.erase(std::unique(z.begin(), z.end()), z.end());
    return z;
}

// ------------------------------------------------------------------ recurrence
// Orthonormal Jacobi polynomials for w(x) = (1-x)^a (1+x)^b:
//   x p_k = be[k+1] p_{k+1} + al[k] p_k + be[k] p_{k-1},  p_0 = mu0^{-1/2}.
struct Rec {
    std::vector<ld> al, be, ibe;        // ibe[k] = 1 / be[k] (k >= 1)
    std::vector<double> al_d, be_d, ibe_d;  // the same, rounded to double
    ld mu0 = 0, sqrt_mu0 = 0;
};

static Rec recurrence(int N, ld a, ld b)
{
    Rec r;
    r.al.resize(N + 1);
    r.be.resize(N + 2);
    const ld ab = a + b;
    for (int k = 0; k <= N; ++k) {
        if (k == 0) {
            r.al[k] = (b - a) / (ab + 2);
        } else {
            ld s = 2 * (ld)k + ab;
            r.al[k] = (b - a) * (b + a) / (s * (s + 2));
        }
    }
    r.be[0] = 0;
    for (int k = 1; k <= N + 1; ++k) {
        if (k == 1) {
            r.be[1] = sqrtl(4 * (1 + a) * (1 + b) / ((ab + 2) * (ab + 2) * (ab + 3)));
        } else {
            ld s = 2 * (ld)k + ab;
            r.be[k] = sqrtl(4 * (ld)k * (k + a) * (k + b) * (k + ab) / (s * s * (s + 1) * (s - 1)));
        }
    }
    r.ibe.assign(N + 2, 0);
    for (int k = 1; k <= N + 1; ++k) r.ibe[k] = 1 / r.be[k];
    r.al_d.assign(r.al.begin(), r.al.end());
    r.be_d.assign(r.be.begin(), r.be.end());
    r.ibe_d.assign(r.ibe.begin(), r.ibe.end());
    r.mu0 = expl((ab + 1) * logl(2.0L) + lgammal(a + 1) + lgammal(b + 1) - lgammal(ab + 2));
    r.sqrt_mu0 = sqrtl(r.mu0);
    return r;
}

// p_n(x), p_{n-1}(x), p_n'(x) and p_{n-1}'(x).
static void eval_top(const Rec &r, int n, ld x, ld &pn, ld &pn1, ld &dpn, ld *dpn1 = nullptr)
{
    ld pm = 0, p = 1 / r.sqrt_mu0, dm = 0, d = 0;
    for (int k = 0; k < n; ++k) {
        ld ip = r.ibe[k + 1];
        ld pnew = ((x - r.al[k]) * p - r.be[k] * pm) * ip;
        ld dnew = ((x - r.al[k]) * d + p - r.be[k] * dm) * ip;
        pm = p; p = pnew;
        dm = d; d = dnew;
    }
    pn = p; pn1 = pm; dpn = d;
    if (dpn1) *dpn1 = dm;
}

// Gauss-Jacobi weight at (an approximation of) a zero of p_n, from the
// Christoffel-Darboux identity  sum_{k<n} p_k^2 = be_n (p_n' p_{n-1} - p_{n-1}' p_n).
// Keeping the second term makes the result insensitive to the last-bit
// error of the zero itself (important near x = +-1, where x = cos t cannot
// resolve the root finer than its own rounding).
static ld weight_at(const Rec &r, int n, ld x)
{
    ld pn, pn1, dpn, dpn1;
    eval_top(r, n, x, pn, pn1, dpn, &dpn1);
    return 1 / (r.be[n] * (dpn * pn1 - dpn1 * pn));
}

// ------------------------------------------------------------------ nodes
// Newton iteration in t on p_n(cos t) from the interior asymptotic zeros
// t_j ~ (j + a/2 - 1/4) pi / (n + (a+b+1)/2); a sign-change scan is the
// fallback when the Newton roots are not n distinct increasing values.
// Double-precision Newton phase for up to 8 roots at once: the recurrence is
// a chain of dependent multiply-adds, so walking 8 independent chains side by
// side keeps the floating-point pipeline busy.  A lane stops when its step
// drops below 1e-11 (conv = 1) or leaves its bracket (conv = 0).
static void newton_double_group(const Rec &r, int n, int cnt, double *t, const double *lo,
                                const double *hi, bool *conv)
{
    constexpr int G = 8;
    bool act[G];
    double x[G];
    for (int i = 0; i < G; ++i) {
        act[i] = i < cnt;
        conv[i] = false;
    }
    const double p0 = (double)(1 / r.sqrt_mu0);
    for (int it = 0; it < 40; ++it) {
        bool any = false;
        for (int i = 0; i < G; ++i) {
            any |= act[i];
            x[i] = (i < cnt) ? std::cos(t[i]) : 0.0;
        }
        if (!any) break;
        double pm[G], p[G], dm[G], d[G];
        for (int i = 0; i < G; ++i) { pm[i] = 0; p[i] = p0; dm[i] = 0; d[i] = 0; }
        for (int k = 0; k < n; ++k) {
            const double ip = r.ibe_d[k + 1], al = r.al_d[k], bk = r.be_d[k];
            for (int i = 0; i < G; ++i) {
                const double xa = x[i] - al;
                const double pn = (xa * p[i] - bk * pm[i]) * ip;
                const double dn = (xa * d[i] + p[i] - bk * dm[i]) * ip;
                pm[i] = p[i]; p[i] = pn;
                dm[i] = d[i]; d[i] = dn;
            }
        }
        for (int i = 0; i < cnt; ++i) {
            if (!act[i]) continue;
            const double fp = -std::sin(t[i]) * d[i];
            if (fp == 0 || !std::isfinite(fp) || !std::isfinite(p[i])) { act[i] = false; continue; }
            const double step = p[i] / fp, tn = t[i] - step;
            if (!(tn > lo[i] && tn < hi[i])) { act[i] = false; continue; }
            t[i] = tn;
            if (std::fabs(step) < 1e-11) { act[i] = false; conv[i] = true; }
        }
    }
}

// Christoffel weights in double for up to 8 roots at once,
// 1 / omega = sum_{k<n} phat_k(x)^2 (a sum of positive terms: no cancellation
// next to x = +-1).  For plans whose tolerance is far above the double
// precision node error.
static void weights_double_group(const Rec &r, int n, int cnt, const double *t, double *w)
{
    constexpr int G = 8;
    const double p0 = (double)(1 / r.sqrt_mu0);
    double x[G], pm[G], p[G], s[G];
    for (int i = 0; i < G; ++i) {
        x[i] = (i < cnt) ? std::cos(t[i]) : 0.0;
        pm[i] = 0; p[i] = p0; s[i] = 0;
    }
    for (int k = 0; k < n; ++k) {
        const double ip = r.ibe_d[k + 1], al = r.al_d[k], bk = r.be_d[k];
        for (int i = 0; i < G; ++i) {
            s[i] += p[i] * p[i];
            const double pn = ((x[i] - al) * p[i] - bk * pm[i]) * ip;
            pm[i] = p[i]; p[i] = pn;
        }
    }
    for (int i = 0; i < cnt; ++i) w[i] = 1.0 / s[i];
}

// One long double Newton step from a root already accurate to double
// precision, returning the Gauss-Jacobi weight as well.  The weight is the
// reciprocal of F(x) = sum_{k<n} p_k(x)^2 = be_n (p_n' p_{n-1} - p_{n-1}' p_n)
// (Christoffel-Darboux), evaluated at the starting point and carried to the
// refined root to first order with F'/F = p_n'' / p_n' + O(p_n), where p_n''
// comes from the Jacobi differential equation
//   (1 - x^2) p'' + (b - a - (a + b + 2) x) p' + n (n + a + b + 1) p = 0.
// One walk of the recurrence gives both the step and the weight; the
// neglected terms are below 1e-20 relative for a starting error near 1e-16.
static bool newton_final(const Rec &r, int n, ld a, ld b, ld &t, ld &omega)
{
    const ld x = cosl(t);
    ld pn, pn1, dpn, dpn1;
    eval_top(r, n, x, pn, pn1, dpn, &dpn1);
    const ld fp = -sinl(t) * dpn;
    if (fp == 0 || !std::isfinite((double)fp)) return false;
    const ld step = pn / fp;
    const ld tn = t - step;
    // x(tn) - x(t) without cancellation
    const ld dx = -2 * sinl((tn + t) / 2) * sinl((tn - t) / 2);
    const ld omx2 = sinl(t) * sinl(t);  // 1 - x^2
    const ld d2 = -((b - a - (a + b + 2) * x) * dpn + n * (n + a + b + 1) * pn) / omx2;
    const ld F = r.be[n] * (dpn * pn1 - dpn1 * pn);
    const ld Fn = F * (1 + dx * d2 / dpn);
    if (!(Fn > 0)) return false;
    t = tn;
    omega = 1 / Fn;
    return fabsl(step) < 1e-9L;
}

static bool newton_root(const Rec &r, int n, ld &t, ld lo, ld hi, bool near = false)
{
    // `near`: t is already within ~1e-11 of the root (double phase), so one
    // step reaches long double accuracy and one more confirms it
    int extra = -1;
    for (int it = 0; it < 60; ++it) {
        ld pn, pn1, dpn;
        eval_top(r, n, cosl(t), pn, pn1, dpn);
        ld fp = -sinl(t) * dpn;
        if (fp == 0) return false;
        ld step = pn / fp;
        ld tn = t - step;
        if (!(tn > lo && tn < hi)) tn = (tn <= lo) ? 0.5L * (t + lo) : 0.5L * (t + hi);
        t = tn;
        if (extra < 0 && fabsl(step) < 1e-14L) extra = near ? 0 : 2;
        if (extra >= 0 && extra-- == 0) return true;
    }
    return false;
}

// refine: finish every root with one long double Newton step (tolerances
// near double rounding); otherwise the double Newton roots and double
// Christoffel-Darboux weights are kept.
static void nodes_ld(const Rec &r, int n, ld a, ld b, std::vector<ld> &t, std::vector<ld> &om, bool refine = true)
{
    t.assign(n, 0);
    om.assign(n, 0);
    const ld N = n + (a + b + 1) / 2;
    const ld cell = kPi / N;
    std::atomic<int> bad(0);
    parallel_for((n + 7) / 8, [&](int g) {
        const int j0 = 8 * g, cnt = std::min(8, n - j0);
        ld tl[8], lol[8], hil[8];
        double td[8], lod[8], hid[8];
        bool conv[8];
        for (int i = 0; i < cnt; ++i) {
            ld tj = (j0 + i + 1 + a / 2 - 0.25L) * cell;
            ld lo = std::max<ld>(0, tj - cell), hi = std::min<ld>(kPi, tj + cell);
            if (tj <= lo || tj >= hi) tj = 0.5L * (lo + hi);
            tl[i] = tj; lol[i] = lo; hil[i] = hi;
            td[i] = (double)tj; lod[i] = (double)lo; hid[i] = (double)hi;
        }
        newton_double_group(r, n, cnt, td, lod, hid, conv);
        double wd[8];
        if (!refine) weights_double_group(r, n, cnt, td, wd);
        for (int i = 0; i < cnt; ++i) {
            if (!refine && conv[i] && wd[i] > 0 && std::isfinite(wd[i])) {
                t[j0 + i] = td[i];
                om[j0 + i] = wd[i];
                continue;
            }
            ld tj = conv[i] ? (ld)td[i] : tl[i];
            ld w = 0;
            if (conv[i] && newton_final(r, n, a, b, tj, w) && tj > lol[i] && tj < hil[i]) {
                t[j0 + i] = tj;
                om[j0 + i] = w;
                continue;
            }
            tj = tl[i];
            if (!newton_root(r, n, tj, lol[i], hil[i])) bad.fetch_add(1);
            t[j0 + i] = tj;
            om[j0 + i] = weight_at(r, n, cosl(tj));
        }
    });
    bool ok = bad.load() == 0;
    for (int j = 0; ok && j < n; ++j) {
        if (!(t[j] > 0 && t[j] < kPi)) ok = false;
        if (j && !(t[j] > t[j - 1] + 1e-6L * cell)) ok = false;
    }
    if (ok) return;
    // fallback: bracket every root by sign changes on a fine grid in t
    const int M = 32 * n + 64;
    std::vector<ld> tg(M), fg(M);
    parallel_for(M, [&](int i) {
        tg[i] = kPi * (i + 0.5L) / M;
        ld pn, pn1, dpn;
        eval_top(r, n, cosl(tg[i]), pn, pn1, dpn);
        fg[i] = pn;
    });
    std::vector<std::pair<ld, ld>> br;
    for (int i = 0; i + 1 < M; ++i)
        if ((fg[i] < 0) != (fg[i + 1] < 0)) br.push_back({tg[i], tg[i + 1]});
    if ((int)br.size() != n) throw std::runtime_error("Gauss-Jacobi node search did not isolate n roots");
    parallel_for(n, [&](int j) {
        ld lo = br[j].first, hi = br[j].second;
        ld tj = 0.5L * (lo + hi);
        // bisection to a small bracket, then Newton
        for (int it = 0; it < 40; ++it) {
            ld pl, p1, d;
            eval_top(r, n, cosl(lo), pl, p1, d);
            ld pm, q1, e;
            eval_top(r, n, cosl(tj), pm, q1, e);
            if ((pl < 0) != (pm < 0)) hi = tj; else lo = tj;
            tj = 0.5L * (lo + hi);
            if (hi - lo < 1e-9L * cell) break;
        }
        if (!newton_root(r, n, tj, lo - cell * 1e-6L, hi + cell * 1e-6L)) bad.fetch_add(1);
        t[j] = tj;
        om[j] = weight_at(r, n, cosl(tj));
    });
}

void gauss_jacobi(int n, double a, double b, std::vector<double> &t, std::vector<double> &x,
                  std::vector<double> &omega)
{
    Rec r = recurrence(n, a, b);
    std::vector<ld> tl, wl;
    nodes_ld(r, n, a, b, tl, wl);
    t.resize(n); x.resize(n); omega.resize(n);
    for (int j = 0; j < n; ++j) {
        t[j] = (double)tl[j];
        x[j] = (double)cosl(tl[j]);
        omega[j] = (double)wl[j];
    }
}

// ------------------------------------------------------------------ companion
// H(x) = PV int (1-s)^a (1+s)^b / (s - x) ds
//      = w(x) log((1-x)/(1+x)) + int_{-1}^{1} (w(s) - w(x)) / (s - x) ds.
// The smooth remainder is split at s = x into two halves.  On each half, with
// v = |s - x|, the integrand is  +-w(x) expm1(Lambda(v)) / v  where Lambda is
// the log of w(s)/w(x) written with log1p so it stays accurate for small v.
// Each half has a power singularity at its far end (+-1) and a nearby one just
// beyond x at distance delta (the other endpoint); it is cut into geometric
// pieces d_{i+1} = 2 d_i + delta graded away from x (Gauss-Legendre 16 on each)
// and a final tanh-sinh piece that reaches the far endpoint.
namespace {
struct QuadTables {
    ld gl_x[16], gl_w[16];
    std::vector<ld> ts_tau, ts_ctau, ts_w;  // tanh-sinh: tau, 1 - tau, weight
    QuadTables()
    {
        Rec r = recurrence(16, 0, 0);
        std::vector<ld> tl, wl;
        nodes_ld(r, 16, 0, 0, tl, wl);
        for (int j = 0; j < 16; ++j) {
            gl_x[j] = cosl(tl[j]);
            gl_w[j] = wl[j];  // Gauss-Legendre weights on [-1, 1]
        }
        // The far-end singularity (ell - v)^e with e close to -1 leaves the
        // transformed integrand decaying only like (1 - tau)^(1 + e); the
        // range |y| <= 8.25 keeps that tail below 1e-20 for e >= -0.99.
        const ld h = 1.0L / 16;
        const int K = 132;
        for (int k = -K; k <= K; ++k) {
            ld y = k * h;
            ld yp = kPi / 2 * sinhl(y);
            ld tau = 1 / (1 + expl(-2 * yp));
            ld ctau = 1 / (1 + expl(2 * yp));
            ld w = h * kPi * coshl(y) * tau * ctau;
            ts_tau.push_back(tau);
            ts_ctau.push_back(ctau);
            ts_w.push_back(w);
        }
    }
};
const QuadTables &quad_tables()
{
    static QuadTables t;
    return t;
}

// integral over v in [0, ell] of expm1(e_far*log((ell-v)/ell) + e_near*log1p(v/delta)) / v,
// in long double (F = ld) or, for plans whose tolerance is far above double
// rounding, in double (F = double): the rank needs the companion only to well
// below the tolerance, and the transform does not depend on it.
template <class F>
F half_integral(F e_far, F e_near, F ell, F delta)
{
    const QuadTables &T = quad_tables();
    auto phi = [&](F v, F ellmv) -> F {
        F lf = (v < F(0.5) * ell) ? std::log1p(-v / ell) : std::log(ellmv / ell);
        F lam = e_far * lf + e_near * std::log1p(v / delta);
        return std::expm1(lam) / v;
    };
    F sum = 0;
    F d = 0;
    for (;;) {
        F nxt = 2 * d + delta;
        if (nxt > F(0.5) * ell) break;
        F c = F(0.5) * (d + nxt), h = F(0.5) * (nxt - d);
        for (int i = 0; i < 16; ++i) {
            F v = c + h * (F)T.gl_x[i];
            sum += h * (F)T.gl_w[i] * phi(v, ell - v);
        }
        d = nxt;
    }
    const F len = ell - d;
    for (size_t k = 0; k < T.ts_tau.size(); ++k) {
        F v = d + len * (F)T.ts_tau[k];
        F ellmv = len * (F)T.ts_ctau[k];
        if (!(v > 0) || !(ellmv > 0)) continue;
        sum += len * (F)T.ts_w[k] * phi(v, ellmv);
    }
    return sum;
}

template <class F>
F hilbert_weight_parts(F omx, F opx, F a, F b)
{
    F wx = std::pow(omx, a) * std::pow(opx, b);
    F right = half_integral<F>(a, b, omx, opx);
    F left = half_integral<F>(b, a, opx, omx);
    return wx * (std::log(omx / opx) + right - left);
}
}  // namespace

long double hilbert_weight(long double x, long double a, long double b)
{
    return hilbert_weight_parts<ld>(1 - x, 1 + x, a, b);
}

// ------------------------------------------------------------------ matrix W B
namespace {
struct Evaluator {
    int n = 0, nu0 = 0, L = 0, Nc = 0;
    double a = 0.0, b = 0.0;
    Rec rec;
    std::vector<ld> x, sw, invpw, q0;  // node, sqrt(omega), 1/(pi w(x)), q_0(x)
    std::vector<int> m;
    std::vector<cd> ph;  // ph[p] = exp(-2 pi i p / L)

    // q_0 at node j.  Plans whose sampled columns come from the phase
    // functions need it only for the sampled rows (lazy_q0): it is computed
    // there from 1 - x_j and 1 + x_j instead of once for every node.
    bool lazy_q0 = false, dbl_q = false;
    std::vector<ld> omx, opx;
    ld q0_at(int j) const
    {
        if (!lazy_q0) return q0[j];
        return (dbl_q ? (ld)hilbert_weight_parts<double>((double)omx[j], (double)opx[j], a, b)
                      : hilbert_weight_parts<ld>(omx[j], opx[j], a, b)) / rec.sqrt_mu0;
    }

    // Walk the p and q recurrences at node j up to degree kmax, calling
    // emit(k, p_k, q_k) for every k (q_k = 0 without with_q).
    template <class F>
    void walk(int j, int kmax, F emit, bool with_q = true) const
    {
        const ld xj = x[j];
        ld pm = 0, p = 1 / rec.sqrt_mu0, qm = 0, q = with_q ? q0_at(j) : 0;
        for (int k = 0; k <= kmax; ++k) {
            emit(k, p, q);
            if (k == kmax) break;
            ld ib = rec.ibe[k + 1];
            ld pn = ((xj - rec.al[k]) * p - rec.be[k] * pm) * ib;
            ld qn = ((xj - rec.al[k]) * q - rec.be[k] * qm + (k == 0 ? rec.sqrt_mu0 : 0)) * ib;
            pm = p; p = pn;
            qm = q; q = qn;
        }
    }
    cd entry(int j, int k, ld p, ld q) const
    {
        int64_t e = ((int64_t)m[j] * k) % L;
        cd z((double)(sw[j] * p), (double)(sw[j] * q * invpw[j]));
        return z * ph[e];
    }
    void row(int j, cd *out) const
    {
        walk(j, n - 1, [&](int k, ld p, ld q) {
            if (k >= nu0) out[k - nu0] = entry(j, k, p, q);
        });
    }
    // Sampled columns in double precision, 8 nodes walked side by side (the
    // recurrence is a dependent chain; independent chains fill the pipeline).
    // Used when the tolerance is far above the double-precision recurrence
    // error (about 1e-14 at these degrees).
    bool dbl_cols = false;
    CMat cols_double(const std::vector<int> &cs) const
    {
        CMat out(n, (int)cs.size());
        const int kmax = nu0 + cs.back();
        const double p0 = (double)(1 / rec.sqrt_mu0), sm0 = (double)rec.sqrt_mu0;
        parallel_for((n + 7) / 8, [&](int g) {
            constexpr int G = 8;
            const int j0 = 8 * g, cnt = std::min(G, n - j0);
            double xx[G], pm[G], p[G], qm[G], q[G];
            for (int i = 0; i < G; ++i) {
                const int j = j0 + std::min(i, cnt - 1);
                xx[i] = (double)x[j];
                pm[i] = 0; p[i] = p0; qm[i] = 0; q[i] = (double)q0[j];
            }
            size_t ci = 0;
            for (int k = 0; k <= kmax; ++k) {
                while (ci < cs.size() && nu0 + cs[ci] == k) {
                    for (int i = 0; i < cnt; ++i) out(j0 + i, (int)ci) = entry(j0 + i, k, p[i], q[i]);
                    ++ci;
                }
                if (k == kmax) break;
                const double ib = rec.ibe_d[k + 1], al = rec.al_d[k], bk = rec.be_d[k];
                const double add = (k == 0) ? sm0 : 0.0;
                for (int i = 0; i < G; ++i) {
                    const double xa = xx[i] - al;
                    const double pn = (xa * p[i] - bk * pm[i]) * ib;
                    const double qn = (xa * q[i] - bk * qm[i] + add) * ib;
                    pm[i] = p[i]; p[i] = pn;
                    qm[i] = q[i]; q[i] = qn;
                }
            }
        });
        return out;
    }
    // columns (degree offsets c = k - nu0), sorted ascending
    // ---- phase-function columns (Section 2.2)
    // The phase grid, each node's panel and barycentric coefficients, its
    // offset from its DFT bin delta_j = t_j - 2 pi m_j / L, and the row scale
    // rs_j = sqrt(omega_j / (w(x_j) sin t_j)) that turns Ptilde + i Qtilde into
    // a row of W B; the data panel's points with their factors
    // sqrt(w sin t), sqrt(sin t / w) / pi and q_0.
    bool phase_cols = false;
    std::unique_ptr<PhaseGrid> grid;
    std::vector<BaryPoint> bp;
    std::vector<double> delta, tn, rs;
    ld dx[PhaseGrid::kPts], dsP[PhaseGrid::kPts], dsQ[PhaseGrid::kPts], dq0[PhaseGrid::kPts];

    void set_phase_data()
    {
        const int D = grid->data;
        for (int i = 0; i < PhaseGrid::kPts; ++i) {
            const ld t = grid->point(D, i);
            const ld sh = sinl(t / 2), ch = cosl(t / 2);
            const ld om = 2 * sh * sh, op = 2 * ch * ch;
            const ld wx = powl(om, (ld)a) * powl(op, (ld)b);
            dx[i] = cosl(t);
            dsP[i] = sqrtl(wx * sinl(t));
            dsQ[i] = sqrtl(sinl(t) / wx) / kPi;
            dq0[i] = hilbert_weight_parts<ld>(om, op, a, b) / rec.sqrt_mu0;
        }
    }
    // Ptilde_k and Qtilde_k at the data panel's points for the ascending
    // degrees degs (P, Q: degs.size() x kPts); with sturm, also the number of
    // sign changes of p_0 .. p_{degs.back()} at each point (the zeros of
    // p_{degs.back()} between that point and t = 0).
    void data_values(const std::vector<int> &degs, std::vector<double> &P, std::vector<double> &Q,
                     int *sturm = nullptr) const
    {
        constexpr int K = PhaseGrid::kPts;
        P.assign(degs.size() * K, 0.0);
        Q.assign(degs.size() * K, 0.0);
        const int kmax = degs.back();
        for (int i = 0; i < K; ++i) {
            ld pm = 0, p = 1 / rec.sqrt_mu0, qm = 0, q = dq0[i];
            int changes = 0;
            ld last = p;
            size_t ci = 0;
            for (int k = 0; k <= kmax; ++k) {
                if (p != 0) {
                    if ((p < 0) != (last < 0)) ++changes;
                    last = p;
                }
                while (ci < degs.size() && degs[ci] == k) {
                    P[ci * K + i] = (double)(dsP[i] * p);
                    Q[ci * K + i] = (double)(dsQ[i] * q);
                    ++ci;
                }
                if (k == kmax) break;
                const ld ib = rec.ibe[k + 1];
                const ld pn = ((dx[i] - rec.al[k]) * p - rec.be[k] * pm) * ib;
                const ld qn = ((dx[i] - rec.al[k]) * q - rec.be[k] * qm + (k == 0 ? rec.sqrt_mu0 : 0)) * ib;
                pm = p; p = pn;
                qm = q; q = qn;
            }
            if (sturm) sturm[i] = changes;
        }
    }
    // Columns (degree offsets cs) from the amplitude and phase of each
    // degree: entry = rs_j sqrt(N) exp(i (k delta_j + (a+b+1)/2 t_j + theta)),
    // i.e. (Ptilde + i Qtilde)(t_j) exp(-2 pi i m_j k / L) with the row scale.
    CMat cols_phase(const std::vector<int> &cs) const
    {
        constexpr int K = PhaseGrid::kPts;
        const int nc = (int)cs.size();
        std::vector<int> degs(nc);
        for (int i = 0; i < nc; ++i) degs[i] = nu0 + cs[i];
        std::vector<double> P, Q;
        data_values(degs, P, Q);
        std::vector<DegreePhase> tab(nc);
        parallel_for(nc, [&](int i) { solve_phase(*grid, degs[i], &P[(size_t)i * K], &Q[(size_t)i * K], tab[i]); });
        const double shift = 0.5 * (a + b + 1.0);
        CMat out(n, nc);
        parallel_for(n, [&](int j) {
            for (int i = 0; i < nc; ++i) {
                double N, th;
                eval_phase(tab[i], bp[j], N, th);
                const double phi = degs[i] * delta[j] + shift * tn[j] + th;
                const double amp = rs[j] * std::sqrt(N);
                out(j, i) = cd(amp * std::cos(phi), amp * std::sin(phi));
            }
        });
        return out;
    }

    CMat cols(const std::vector<int> &cs) const
    {
        if (phase_cols && !cs.empty()) return cols_phase(cs);
        if (dbl_cols && !cs.empty()) return cols_double(cs);
        CMat out(n, (int)cs.size());
        if (cs.empty()) return out;
        int kmax = nu0 + cs.back();
        parallel_for(n, [&](int j) {
            size_t ci = 0;
            walk(j, kmax, [&](int k, ld p, ld q) {
                while (ci < cs.size() && nu0 + cs[ci] == k) {
                    out(j, (int)ci) = entry(j, k, p, q);
                    ++ci;
                }
            });
        });
        return out;
    }
    // Sampled rows in double precision (same tolerance condition as
    // cols_double).  Blocks of up to 64 rows walk the recurrence in lock step,
    // one degree at a time, so every degree fills a contiguous piece of its
    // column and the per-row updates run as plain vector loops.
    CMat rows_double(const std::vector<int> &rs) const
    {
        const int nr = (int)rs.size();
        CMat out(nr, Nc);
        constexpr int RB = 64;
        const double p0 = (double)(1 / rec.sqrt_mu0), sm0 = (double)rec.sqrt_mu0;
        const int nblk = (nr + RB - 1) / RB;
        parallel_for(nblk, [&](int blk) {
            const int i0 = blk * RB, cnt = std::min(RB, nr - i0);
            double xx[RB], pm[RB], p[RB], qm[RB], q[RB], sp[RB], sq[RB];
            int e[RB], mm[RB];
            for (int i = 0; i < cnt; ++i) {
                const int j = rs[i0 + i];
                xx[i] = (double)x[j];
                pm[i] = 0; p[i] = p0; qm[i] = 0; q[i] = (double)q0_at(j);
                sp[i] = (double)sw[j];
                sq[i] = (double)(sw[j] * invpw[j]);
                mm[i] = m[j];
                e[i] = (int)(((int64_t)m[j] * nu0) % L);
            }
            for (int k = 0; k < n; ++k) {
                if (k >= nu0) {
                    cd *col = &out.a[(size_t)(k - nu0) * nr + i0];
                    for (int i = 0; i < cnt; ++i) {
                        const cd w = ph[e[i]];
                        const double zr = sp[i] * p[i], zi = sq[i] * q[i];
                        col[i] = cd(zr * w.real() - zi * w.imag(), zr * w.imag() + zi * w.real());
                        e[i] += mm[i];
                        e[i] -= (e[i] >= L) ? L : 0;
                    }
                }
                if (k == n - 1) break;
                const double ib = rec.ibe_d[k + 1], al = rec.al_d[k], bk = rec.be_d[k];
                const double add = (k == 0) ? sm0 : 0.0;
                for (int i = 0; i < cnt; ++i) {
                    const double xa = xx[i] - al;
                    const double pn = (xa * p[i] - bk * pm[i]) * ib;
                    const double qn = (xa * q[i] - bk * qm[i] + add) * ib;
                    pm[i] = p[i]; p[i] = pn;
                    qm[i] = q[i]; q[i] = qn;
                }
            }
        });
        return out;
    }
    CMat rows(const std::vector<int> &rs) const
    {
        if (dbl_cols && !rs.empty() && Nc > 0) return rows_double(rs);
        CMat out((int)rs.size(), Nc);
        parallel_for((int)rs.size(), [&](int i) {
            std::vector<cd> r(Nc);
            row(rs[i], r.data());
            for (int c = 0; c < Nc; ++c) out(i, c) = r[c];
        });
        return out;
    }
};
}  // namespace

static void rsvd(const Evaluator &E, double tol, const PlanOptions &opt, uint64_t seed, AxisPlan &ax)
{
    const int Nr = E.n, Nc = E.Nc;
    const int rmax = std::min(Nr, Nc);
    int r = std::min(rmax, std::max(4, (int)std::ceil(2.0 * std::log2((double)E.n))));
    Rng rng(seed);
    // the a-posteriori check: every row up to 512 rows, else 512 sampled rows
    const bool all_rows = Nr <= 512;
    std::vector<int> check_rows;
    if (all_rows) {
        check_rows.resize(Nr);
        std::iota(check_rows.begin(), check_rows.end(), 0);
    } else {
        check_rows = sample(rng, Nr, 512, {});
    }
    const CMat Zc = E.rows(check_rows);
    double zc2 = 0.0;
    for (const cd &z : Zc.a) zc2 += std::norm(z);

    // Relative Frobenius error of U0 diag(s) Vh on the check rows, truncated
    // to the first `keep` terms and with all rk terms, in one pass over the
    // columns (each column of the check rows and of Vh is contiguous).  The
    // per-chunk partial sums are added in chunk order, so the result does not
    // depend on the thread count.
    auto rel_errors = [&](const CMat &U0, const std::vector<double> &s, const CMat &Vh, int rk, int keep) {
        const int nchk = (int)check_rows.size();
        // U0 diag(s) on the check rows, real and imaginary parts apart (plain
        // real loops below)
        std::vector<double> Cr((size_t)nchk * rk), Ci((size_t)nchk * rk);
        for (int l = 0; l < rk; ++l)
            for (int i = 0; i < nchk; ++i) {
                const cd z = U0(check_rows[i], l) * s[l];
                Cr[(size_t)l * nchk + i] = z.real();
                Ci[(size_t)l * nchk + i] = z.imag();
            }
        auto norm2 = [&](const double *xr, const double *xi) {
            double e0 = 0.0, e1 = 0.0;
            for (int i = 0; i < nchk; ++i) {
                e0 += xr[i] * xr[i];
                e1 += xi[i] * xi[i];
            }
            return e0 + e1;
        };
        constexpr int kChunk = 64;
        const int nchunk = (Nc + kChunk - 1) / kChunk;
        std::vector<double> pk(nchunk, 0.0), pf(nchunk, 0.0);
        parallel_for(nchunk, [&](int ch) {
            std::vector<double> rr(nchk), ri(nchk);
            double ek = 0.0, ef = 0.0;
            const int c1 = std::min(Nc, (ch + 1) * kChunk);
            for (int c = ch * kChunk; c < c1; ++c) {
                for (int i = 0; i < nchk; ++i) {
                    rr[i] = Zc(i, c).real();
                    ri[i] = Zc(i, c).imag();
                }
                for (int l = 0; l < rk; ++l) {
                    if (l == keep) ek += norm2(rr.data(), ri.data());
                    const double vr = Vh(l, c).real(), vi = Vh(l, c).imag();
                    const double *cr = &Cr[(size_t)l * nchk], *ci = &Ci[(size_t)l * nchk];
                    for (int i = 0; i < nchk; ++i) {
                        rr[i] -= cr[i] * vr - ci[i] * vi;
                        ri[i] -= cr[i] * vi + ci[i] * vr;
                    }
                }
                const double e = norm2(rr.data(), ri.data());
                ef += e;
                if (keep >= rk) ek += e;
            }
            pk[ch] = ek;
            pf[ch] = ef;
        });
        double e2k = 0.0, e2f = 0.0;
        for (int ch = 0; ch < nchunk; ++ch) {
            e2k += pk[ch];
            e2f += pf[ch];
        }
        return std::make_pair(std::sqrt(e2k / zc2), std::sqrt(e2f / zc2));
    };

    for (int round = 0;; ++round) {
        ax.rsvd_rounds = round + 1;
        const int qr = std::max(1, opt.oversample) * r;
        std::vector<int> Pcol, Prow;
        CMat ZJ;
        std::vector<int> J;
        for (int it = 0; it < std::max(1, opt.iterations); ++it) {
            // step 2: sampled rows plus the current important rows; pivoted QR
            std::vector<int> I = merged(sample(rng, Nr, qr, Prow), Prow);
            CMat ZI = E.rows(I);
            std::vector<int> perm = pivoted_qr(ZI, r, nullptr);
            Pcol.assign(perm.begin(), perm.begin() + std::min<int>(r, (int)perm.size()));
            std::sort(Pcol.begin(), Pcol.end());
            // step 3: sampled columns plus the important columns; pivoted LQ
            J = merged(sample(rng, Nc, qr, Pcol), Pcol);
            ZJ = E.cols(J);
            perm = pivoted_qr(adjoint(ZJ), r, nullptr);
            Prow.assign(perm.begin(), perm.begin() + std::min<int>(r, (int)perm.size()));
            std::sort(Prow.begin(), Prow.end());
        }
        const int rc = (int)Pcol.size(), rr = (int)Prow.size();
        // step 5: orthonormal bases of the important columns and rows
        CMat Zpc(Nr, rc);
        for (int i = 0; i < rc; ++i) {
            int pos = (int)(std::lower_bound(J.begin(), J.end(), Pcol[i]) - J.begin());
            for (int j = 0; j < Nr; ++j) Zpc(j, i) = ZJ(j, pos);
        }
        CMat Qcol, Qrow;
        pivoted_qr(Zpc, rc, &Qcol);
        CMat Zpr = E.rows(Prow);
        pivoted_qr(adjoint(Zpr), rr, &Qrow);
        // step 6: middle matrix by least squares on extra sampled rows/columns
        std::vector<int> J2 = merged(Pcol, sample(rng, Nc, qr, Pcol));
        std::vector<int> I2 = merged(Prow, sample(rng, Nr, qr, Prow));
        CMat ZI2 = E.rows(I2);
        CMat ZIJ((int)I2.size(), (int)J2.size());
        for (int i = 0; i < (int)I2.size(); ++i)
            for (int c = 0; c < (int)J2.size(); ++c) ZIJ(i, c) = ZI2(i, J2[c]);
        CMat A1((int)I2.size(), rc);
        for (int i = 0; i < (int)I2.size(); ++i)
            for (int l = 0; l < rc; ++l) A1(i, l) = Qcol(I2[i], l);
        CMat B1(rr, (int)J2.size());
        for (int l = 0; l < rr; ++l)
            for (int c = 0; c < (int)J2.size(); ++c) B1(l, c) = std::conj(Qrow(J2[c], l));
        CMat M = matmul(matmul(pinv(A1), ZIJ), pinv(B1));
        // step 7: SVD of the middle matrix
        CMat UM, VM;
        std::vector<double> s;
        svd(M, UM, s, VM);
        CMat U0 = matmul(Qcol, UM);
        CMat Vh = matmul(adjoint(VM), adjoint(Qrow));
        const int rk = (int)s.size();
        // truncate: drop the tail whose Frobenius mass is below tol/2
        double fro2 = 0.0;
        for (double v : s) fro2 += v * v;
        int keep = rk;
        double tail2 = 0.0;
        while (keep > 0) {
            double t2 = tail2 + s[keep - 1] * s[keep - 1];
            if (std::sqrt(t2 / std::max(fro2, 1e-300)) > 0.5 * tol) break;
            tail2 = t2;
            --keep;
        }
        const auto errs = rel_errors(U0, s, Vh, rk, keep);
        const double err_full = errs.second;
        bool last = (r >= rmax);
        if (err_full <= 0.5 * tol || last) {
            double err = errs.first;
            if (err > tol && keep < rk) {
                keep = rk;
                err = err_full;
            }
            if (err > tol && !last) {
                r = std::min(rmax, (int)std::ceil(1.5 * r) + 2);
                continue;
            }
            ax.rank = keep;
            ax.rel_err = err;
            ax.fro = std::sqrt(zc2 * (all_rows ? 1.0 : (double)Nr / check_rows.size()));
            ax.U.assign((size_t)keep * Nr, cd(0.0, 0.0));
            ax.V.assign((size_t)keep * ax.L, cd(0.0, 0.0));
            for (int l = 0; l < keep; ++l) {
                double sh = std::sqrt(s[l]);
                for (int j = 0; j < Nr; ++j) ax.U[(size_t)l * Nr + j] = U0(j, l) * sh;
                for (int c = 0; c < Nc; ++c) ax.V[(size_t)l * ax.L + E.nu0 + c] = Vh(l, c) * sh;
            }
            if (err > tol)
                throw std::runtime_error("randomized SVD did not reach the requested tolerance");
            return;
        }
        r = std::min(rmax, (int)std::ceil(1.5 * r) + 2);
    }
}

// ------------------------------------------------------------------ build
static void check_axis_args(int n, double a, double b, double tol, const PlanOptions &opt)
{
    if (n < 1 || n > (1 << 14)) throw std::invalid_argument("n must be in [1, 16384]");
    if (!(a > -1.0) || !(b > -1.0) || !(a < 1.0) || !(b < 1.0))
        throw std::invalid_argument("a and b must lie in (-1, 1)");
    if (!(tol >= 1e-14) || !(tol <= 1e-2)) throw std::invalid_argument("tol must lie in [1e-14, 1e-2]");
    if (opt.nu0 < 1 || opt.nu0 > kMaxNu0) throw std::invalid_argument("nu0 must lie in [1, 64]");
    if (opt.kind != 1 && opt.kind != 2) throw std::invalid_argument("kind must be 1 (first) or 2 (second)");
    if (opt.planner < 0 || opt.planner > 2) throw std::invalid_argument("planner must be 0, 1 or 2");
}

// Sizes, direct-block width and seed of an axis; the evaluator's shape.
static void start_axis(AxisPlan &ax, Evaluator &E, int n, double a, double b, double tol, const PlanOptions &opt)
{
    ax = AxisPlan();
    ax.n = n; ax.a = a; ax.b = b; ax.tol = tol;
    int L = 64;
    while (L < n) L *= 2;
    ax.L = L;
    // dense (every degree in the direct block) below the crossover, up to the
    // longest line the matrix-core pass takes
    ax.nu0 = (n < opt.dense_below && n <= 1024) ? n : std::min(opt.nu0, n);
    ax.seed = opt.seed ? opt.seed : mix_key(n, a, b, tol);
    ax.kind = opt.kind;
    E.n = n; E.nu0 = ax.nu0; E.L = L; E.Nc = n - ax.nu0;
    E.a = a; E.b = b;
    E.dbl_cols = tol >= 1e-10;
    // double quadrature only where the weight's exponents are mild: near -1
    // the tanh-sinh tail of the far-end singularity overflows double range
    E.dbl_q = E.dbl_cols && a > -0.5 && b > -0.5;
    E.rec = recurrence(n + 1, a, b);
    E.x.resize(n); E.sw.resize(n); E.invpw.resize(n); E.q0.resize(n); E.m.resize(n);
    ax.t.resize(n); ax.x.resize(n); ax.omega.resize(n); ax.bins.resize(n);
}

// Phase functions (Section 2.2) give the nodes, the weights and the sampled
// columns of uniform plans for |a|, |b| < 1/2 (the range Section 2.2 treats)
// at tolerances of 1e-8 and looser: the tables carry the phase to about
// 1e-14 lam absolute, so the nodes to about 1e-13 and the entries to about
// 1e-9 at n = 16384, an order below such a tolerance (the recurrence stays for
// the sampled rows and the direct block).  Planner 1 never uses them,
// planner 2 wherever allowed, planner 0 (automatic) from kPhaseAuto points
// on, where they are the faster way (measured crossover near 1024).
constexpr int kPhaseAuto = 1024;
constexpr int kPhaseMin = 64;
static bool phase_allowed(int n, double a, double b, double tol, const PlanOptions &opt)
{
    if (opt.planner == 1 || n < kPhaseMin || !(tol >= 1e-8)) return false;
    if (!(std::fabs(a) < 0.5) || !(std::fabs(b) < 0.5)) return false;
    if (n - std::min(opt.nu0, n) > 0 && opt.nu0 < 27) return false;  // the tables start at degree 27
    return opt.planner == 2 || n >= kPhaseAuto;
}

// Nodes and weights from the phase of degree n: P~_n = M cos psi vanishes
// where psi = pi/2 (mod pi), psi increases, so the j-th node solves
//   psi(t) = psi(t_s) + g + (j - K) pi,   g = (pi/2 - psi(t_s)) mod pi,
// with K the number of nodes below a data point t_s (the sign changes of
// p_0 .. p_n there, by the Sturm property of orthogonal polynomials).
// Newton on the interpolated phase; the Gauss-Jacobi weight in t is
// pi / psi'(t_j) = pi N(t_j) / W (so omega_j = that times w(x_j) sin t_j).
// Returns false (and the caller uses the recurrence) if any node fails to
// converge inside the grid, the nodes do not increase, or P~_n computed by the
// recurrence at three of them is not small.
static bool phase_nodes(const Evaluator &E, int n, std::vector<ld> &tl, std::vector<ld> &wl)
{
    constexpr int K = PhaseGrid::kPts;
    const PhaseGrid &g = *E.grid;
    std::vector<double> P, Q;
    int sturm[K];
    E.data_values(std::vector<int>{n}, P, Q, sturm);
    DegreePhase ph;
    solve_phase(g, n, P.data(), Q.data(), ph);
    // a data point where P~_n is well away from zero (its zero count is then sure)
    int is = -1;
    for (int i = K / 2; i < K - 1 && is < 0; ++i)
        if (std::fabs(P[i]) > 0.25 * std::sqrt(P[i] * P[i] + Q[i] * Q[i])) is = i;
    if (is < 0) return false;
    const double lam = ph.lam, W = 2.0 * lam / (double)kPi;
    const double ts = g.point(g.data, is);
    const BaryPoint bs = bary_point(g, ts);
    double Ns, ths;
    eval_phase(ph, bs, Ns, ths);
    // psi(t_s) mod pi in long double (lam t_s reaches lam pi / 2)
    const ld psis = (ld)lam * (ld)ts + (ld)ths;
    const ld g0 = fmodl(fmodl(kPi / 2 - psis, kPi) + kPi, kPi);
    const int Kz = sturm[is];
    tl.assign(n, 0);
    wl.assign(n, 0);
    std::atomic<int> bad(0);
    const double lo = g.ends.front(), hi = g.ends.back();
    parallel_for(n, [&](int j) {
        // lam (t - t_s) + theta(t) = R_j
        const double R = (double)((ld)ths + g0 + (ld)(j - Kz) * kPi);
        double t = ts + (R - ths) / lam;
        bool conv = false;
        for (int it = 0; it < 40; ++it) {
            t = std::min(hi, std::max(lo, t));
            const BaryPoint bpt = bary_point(g, t);
            double N, th;
            eval_phase(ph, bpt, N, th);
            const double f = lam * (t - ts) + th - R;
            const double dt = f / (W / N);
            t -= dt;
            if (std::fabs(dt) <= 1e-15 * std::max(1.0, t)) {
                conv = t > lo && t < hi;
                break;
            }
        }
        if (!conv) {
            bad.fetch_add(1);
            return;
        }
        const BaryPoint bpt = bary_point(g, t);
        double N, th;
        eval_phase(ph, bpt, N, th);
        const ld tj = t;
        const ld sh = sinl(tj / 2), ch = cosl(tj / 2);
        const ld wsin = powl(2 * sh * sh, (ld)E.a) * powl(2 * ch * ch, (ld)E.b) * sinl(tj);
        tl[j] = tj;
        wl[j] = (ld)kPi * (ld)N / (ld)W * wsin;
    });
    if (bad.load()) return false;
    for (int j = 1; j < n; ++j)
        if (!(tl[j] > tl[j - 1])) return false;
    // spot checks with the recurrence: P~_n(t_j) ~ 0 relative to the amplitude
    for (int j : {0, n / 2, n - 1}) {
        ld pn, pn1, dpn;
        eval_top(E.rec, n, cosl(tl[j]), pn, pn1, dpn);
        const ld sh = sinl(tl[j] / 2), ch = cosl(tl[j] / 2);
        const ld amp = sqrtl(powl(2 * sh * sh, (ld)E.a) * powl(2 * ch * ch, (ld)E.b) * sinl(tl[j]));
        const BaryPoint bpt = bary_point(g, (double)tl[j]);
        double N, th;
        eval_phase(ph, bpt, N, th);
        if (!(fabsl(amp * pn) <= 1e-8L * sqrtl((ld)N))) return false;
    }
    return true;
}

// Per-point values at angle t with row scale sw: the point, its bin
// m = [t L / 2 pi] (eq. (45)), 1 / (pi w(x)) and q_0(x) for the companion.
static void set_point(AxisPlan &ax, Evaluator &E, int j, ld t, ld sw, ld om)
{
    const ld xj = cosl(t);
    const ld sh = sinl(t / 2), ch = cosl(t / 2);
    const ld omx = 2 * sh * sh, opx = 2 * ch * ch;  // 1 - x, 1 + x without cancellation
    const ld wx = powl(omx, (ld)ax.a) * powl(opx, (ld)ax.b);
    E.x[j] = xj;
    E.sw[j] = sw;
    E.invpw[j] = 1 / (kPi * wx);
    E.m[j] = (int)llrintl(t * ax.L / (2 * kPi));
    ax.t[j] = (double)t;
    ax.x[j] = (double)xj;
    ax.omega[j] = (double)om;
    ax.bins[j] = E.m[j];
    if (E.phase_cols) {
        E.bp[j] = bary_point(*E.grid, (double)t);
        E.delta[j] = (double)(t - 2 * kPi * E.m[j] / ax.L);
        E.tn[j] = (double)t;
        E.rs[j] = (double)(sw / sqrtl(wx * sinl(t)));
    }
    if (E.lazy_q0) {
        E.omx[j] = omx;
        E.opx[j] = opx;
    } else if (E.Nc > 0 || ax.kind == 2) {
        E.q0[j] = (E.dbl_q ? (ld)hilbert_weight_parts<double>((double)omx, (double)opx, ax.a, ax.b)
                           : hilbert_weight_parts<ld>(omx, opx, ax.a, ax.b)) / E.rec.sqrt_mu0;
    }
}

// Everything after the points: bin table, direct block, DFT phases and the
// randomized factorization of the low-rank part.
static void finish_axis(AxisPlan &ax, Evaluator &E, const PlanOptions &opt)
{
    const int n = ax.n, L = ax.L;
    // bins are non-decreasing (points ascend in t); CSR over m = 0 .. L/2
    const int nb = L / 2 + 1;
    ax.binptr.assign(nb + 1, 0);
    for (int j = 0; j < n; ++j) {
        if (ax.bins[j] < 0 || ax.bins[j] > L / 2) throw std::runtime_error("bin out of range");
        if (j && ax.bins[j] < ax.bins[j - 1]) throw std::runtime_error("bins not monotone");
        ax.binptr[ax.bins[j] + 1]++;
    }
    ax.max_per_bin = 0;
    for (int m = 0; m < nb; ++m) {
        ax.max_per_bin = std::max(ax.max_per_bin, ax.binptr[m + 1]);
        ax.binptr[m + 1] += ax.binptr[m];
    }
    // direct block: the low degrees of the first-kind functions, or of the
    // second-kind ones (the imaginary part of W B before the DFT phase)
    ax.WV.assign((size_t)ax.nu0 * n, 0.0);
    const bool second = ax.kind == 2;
    parallel_for(n, [&](int j) {
        E.walk(j, ax.nu0 - 1, [&](int k, ld p, ld q) {
            ax.WV[(size_t)k * n + j] = (double)(second ? E.sw[j] * q * E.invpw[j] : E.sw[j] * p);
        }, second);
    });
    // DFT phase table of eq. (45): exp(-2 pi i p / L), exact integer phase
    E.ph.resize(L);
    for (int p = 0; p < L; ++p) {
        ld ang = -2 * kPi * p / L;
        E.ph[p] = cd((double)cosl(ang), (double)sinl(ang));
    }
    if (E.Nc > 0)
        rsvd(E, ax.tol, opt, ax.seed, ax);
    // second kind: Im(u y) = Re((-i u) y), so the same kernels apply the
    // second-kind transform once u is turned by -i (forward and transpose)
    if (second)
        for (cd &z : ax.U) z = cd(z.imag(), -z.real());
}

void build_axis(AxisPlan &ax, int n, double a, double b, double tol, const PlanOptions &opt)
{
    check_axis_args(n, a, b, tol, opt);
    Evaluator E;
    start_axis(ax, E, n, a, b, tol, opt);
    std::vector<ld> tl, wl;
    bool phase = phase_allowed(n, a, b, tol, opt);
    if (phase) {
        E.grid.reset(new PhaseGrid(n, a, b));
        E.set_phase_data();
        phase = phase_nodes(E, n, tl, wl);
    }
    // double-precision nodes and weights are kept at tolerances of 1e-7 and
    // looser: their error (weights to about 3e-17 n^2 relative, from the
    // double x next to +-1) stays two orders below such a tolerance
    if (!phase) nodes_ld(E.rec, n, a, b, tl, wl, tol < 1e-7);
    // sampled columns from the phase tables when every node lies on the grid
    if (phase && E.Nc > 0) {
        bool inside = true;
        for (int j = 0; j < n; ++j) inside = inside && E.grid->panel_of((double)tl[j]) >= 0;
        if (inside) {
            E.phase_cols = true;
            E.lazy_q0 = ax.kind == 1;
            E.bp.resize(n); E.delta.resize(n); E.tn.resize(n); E.rs.resize(n);
            if (E.lazy_q0) { E.omx.resize(n); E.opx.resize(n); }
        }
    }
    ax.planner = phase ? 2 : 1;
    // uniform transform: rows weighted by sqrt(omega_j) (Section 3.1, eq. (37))
    parallel_for(n, [&](int j) { set_point(ax, E, j, tl[j], sqrtl(wl[j]), wl[j]); });
    finish_axis(ax, E, opt);
}

void build_axis_points(AxisPlan &ax, int n, const double *t, double a, double b, double tol,
                       const PlanOptions &opt)
{
    check_axis_args(n, a, b, tol, opt);
    if (!t) throw std::invalid_argument("null point array");
    for (int j = 0; j < n; ++j) {
        if (!(t[j] > 0.0) || !(t[j] < 3.14159265358979323846)) throw std::invalid_argument("points must lie in (0, pi)");
        if (j && !(t[j] >= t[j - 1])) throw std::invalid_argument("points must be non-decreasing");
    }
    Evaluator E;
    start_axis(ax, E, n, a, b, tol, opt);
    ax.points = true;
    // nonuniform transform: the rows are Ptilde_k(t_j) themselves, no
    // quadrature weights (Section 3.1): Ptilde_k(t) = sqrt(w(x) sin t) phat_k(x)
    parallel_for(n, [&](int j) {
        const ld tj = t[j];
        const ld sh = sinl(tj / 2), ch = cosl(tj / 2);
        const ld wsin = powl(2 * sh * sh, (ld)a) * powl(2 * ch * ch, (ld)b) * sinl(tj);
        set_point(ax, E, j, tj, sqrtl(wsin), 0);
    });
    finish_axis(ax, E, opt);
}

void exact_entries(const AxisPlan &ax, int count, const int *rows, const int *degs, cd *out)
{
    Rec rec = recurrence(ax.n + 1, ax.a, ax.b);
    for (int i = 0; i < count; ++i) {
        int j = rows[i], k = degs[i];
        if (j < 0 || j >= ax.n || k < 0 || k >= ax.n) throw std::invalid_argument("entry index out of range");
        ld t = ax.t[j];
        ld xj = cosl(t);
        ld sh = sinl(t / 2), ch = cosl(t / 2);
        ld omx = 2 * sh * sh, opx = 2 * ch * ch;
        ld wx = powl(omx, (ld)ax.a) * powl(opx, (ld)ax.b);
        ld q = hilbert_weight_parts<ld>(omx, opx, ax.a, ax.b) / rec.sqrt_mu0;
        ld pm = 0, p = 1 / rec.sqrt_mu0, qm = 0;
        for (int kk = 0; kk < k; ++kk) {
            ld ib = rec.ibe[kk + 1];
            ld pn = ((xj - rec.al[kk]) * p - rec.be[kk] * pm) * ib;
            ld qn = ((xj - rec.al[kk]) * q - rec.be[kk] * qm + (kk == 0 ? rec.sqrt_mu0 : 0)) * ib;
            pm = p; p = pn;
            qm = q; q = qn;
        }
        ld sw = ax.points ? sqrtl(wx * sinl(t)) : sqrtl((ld)ax.omega[j]);
        int64_t e = ((int64_t)ax.bins[j] * k) % ax.L;
        ld ang = -2 * kPi * e / ax.L;
        cd z((double)(sw * p), (double)(sw * q / (kPi * wx)));
        out[i] = z * cd((double)cosl(ang), (double)sinl(ang));
    }
}

// ------------------------------------------------------------------ packing
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t layout_axis(AxisPlan &ax, size_t base, int precs)
{
    size_t o = align256(base);
    const size_t n = ax.n, L = ax.L, r = ax.rank, nu = ax.nu0;
    const bool f64 = precs & kPackF64, f32 = precs & kPackF32;
    auto sec = [&](size_t &off, bool present, size_t bytes) {
        if (!present) {
            off = kAbsent;
            return;
        }
        off = o;
        o = align256(o + bytes);
    };
    sec(ax.off_tw64, f64, L * 16);
    sec(ax.off_tw32, f32, L * 8);
    sec(ax.off_bins, true, n * 4);
    sec(ax.off_binptr, true, (L / 2 + 2) * 4);
    sec(ax.off_wv64, f64, nu * n * 8);
    sec(ax.off_wv32, f32, nu * n * 4);
    sec(ax.off_u64, f64, r * n * 16);
    sec(ax.off_u32, f32, r * n * 8);
    sec(ax.off_v64, f64, r * L * 16);
    sec(ax.off_v32, f32, r * L * 8);
    ax.bytes = o - base;
    return o;
}

void pack_axis(const AxisPlan &ax, unsigned char *blob)
{
    const int n = ax.n, L = ax.L, r = ax.rank, nu = ax.nu0;
    const bool f64 = ax.off_tw64 != kAbsent, f32 = ax.off_tw32 != kAbsent;
    for (int p = 0; p < L; ++p) {
        // DFT twiddles of eq. (47): exp(+2 pi i p / L)
        ld ang = 2 * kPi * p / L;
        ld c = cosl(ang), s = sinl(ang);
        if (f64) {
            double *tw64 = (double *)(blob + ax.off_tw64);
            tw64[2 * p] = (double)c; tw64[2 * p + 1] = (double)s;
        }
        if (f32) {
            float *tw32 = (float *)(blob + ax.off_tw32);
            tw32[2 * p] = (float)c; tw32[2 * p + 1] = (float)s;
        }
    }
    std::memcpy(blob + ax.off_bins, ax.bins.data(), (size_t)n * 4);
    int32_t *bp = (int32_t *)(blob + ax.off_binptr);
    for (int m = 0; m < L / 2 + 2; ++m) bp[m] = (m < (int)ax.binptr.size()) ? ax.binptr[m] : n;
    for (size_t i = 0; i < (size_t)nu * n; ++i) {
        if (f64) ((double *)(blob + ax.off_wv64))[i] = ax.WV[i];
        if (f32) ((float *)(blob + ax.off_wv32))[i] = (float)ax.WV[i];
    }
    for (size_t i = 0; i < (size_t)r * n; ++i) {
        if (f64) {
            double *u64 = (double *)(blob + ax.off_u64);
            u64[2 * i] = ax.U[i].real(); u64[2 * i + 1] = ax.U[i].imag();
        }
        if (f32) {
            float *u32 = (float *)(blob + ax.off_u32);
            u32[2 * i] = (float)ax.U[i].real(); u32[2 * i + 1] = (float)ax.U[i].imag();
        }
    }
    for (size_t i = 0; i < (size_t)r * L; ++i) {
        if (f64) {
            double *v64 = (double *)(blob + ax.off_v64);
            v64[2 * i] = ax.V[i].real(); v64[2 * i + 1] = ax.V[i].imag();
        }
        if (f32) {
            float *v32 = (float *)(blob + ax.off_v32);
            v32[2 * i] = (float)ax.V[i].real(); v32[2 * i + 1] = (float)ax.V[i].imag();
        }
    }
}

}  // namespace jt
