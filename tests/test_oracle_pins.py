"""Pins for the oracle: checks against facts fixed by the paper and by mathematics,
never against the oracle's own formulas retyped.

* a = b = -1/2: Chebyshev-T special case; A is the orthonormal DCT-III
  (independent library routine: scipy.fft.dct).
* a = b = +1/2: Chebyshev-U special case; A is the orthonormal DST-I.
* brute force at tiny n with mpmath (40 digits): nodes bracketed by sign
  changes of the explicit finite-sum P_n^(a,b), weights from the classical
  derivative formula, norms from the Gamma-function closed form.
* quadrature exactness (eq. (2): exact for degree <= 2n-1) against adaptive
  algebraic-weight integration (scipy QAWS), which pins the measure, including
  which endpoint carries a and which carries b.
* orthogonality of W J (Section 3.1) at the benchmark sizes and the
  forward-inverse identity.
* the Kronecker axis convention (eqs. (54), (59)) against numpy.kron.
* planted mistakes (swapped a/b, reversed node order) must fail the pins.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.fft
from scipy import integrate


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 2, 8, 64, 1000])
def test_chebyshev_t_is_dct3(orc, n):
    A, x, w = orc.matrix(n, -0.5, -0.5)
    j = np.arange(1, n + 1)
    np.testing.assert_allclose(x, np.cos((2 * j - 1) * np.pi / (2 * n)), rtol=0, atol=1e-15)
    # the endpoint weights amplify the ~1e-19 node error of x-space long double
    # arithmetic by ~1e5 (their Christoffel function is steep there)
    np.testing.assert_allclose(w, np.full(n, np.pi / n), rtol=3e-14, atol=0)
    al = np.random.default_rng(1).standard_normal(n)
    ref = scipy.fft.dct(al, type=3, norm="ortho")
    assert np.abs(A @ al - ref).max() <= 5e-14 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n", [1, 3, 8, 64, 1000])
def test_chebyshev_u_is_dst1(orc, n):
    A, x, w = orc.matrix(n, 0.5, 0.5)
    j = np.arange(1, n + 1)
    np.testing.assert_allclose(x, np.cos(j * np.pi / (n + 1)), rtol=0, atol=1e-15)
    al = np.random.default_rng(2).standard_normal(n)
    ref = scipy.fft.dst(al, type=1, norm="ortho")
    assert np.abs(A @ al - ref).max() <= 5e-14 * max(1.0, np.abs(ref).max())


# ------------------------------------------------------------ mpmath brute force
def _mp_matrix(n, a, b, dps=40):
    """Dense A for tiny n from explicit Jacobi polynomials in multiprecision."""
    with mp.workdps(dps):
        a_, b_ = mp.mpf(a), mp.mpf(b)

        def jac(k, al, be, x):
            # explicit finite sum: P_k^(al,be)(x) =
            #   sum_s C(k+al, k-s) C(k+be, s) ((x-1)/2)^s ((x+1)/2)^(k-s)
            xm, xp = (x - 1) / 2, (x + 1) / 2
            return mp.fsum(mp.binomial(k + al, k - s) * mp.binomial(k + be, s)
                           * xm ** s * xp ** (k - s) for s in range(k + 1))

        def pn(t):
            return jac(n, a_, b_, mp.cos(t))

        m = 40 * n
        grid = [mp.pi * i / m for i in range(1, m)]
        vals = [pn(t) for t in grid]
        ts = []
        for i in range(len(grid) - 1):
            if vals[i] == 0:
                ts.append(grid[i])
            elif vals[i] * vals[i + 1] < 0:
                ts.append(mp.findroot(pn, (grid[i], grid[i + 1]), solver="anderson"))
        assert len(ts) == n, (len(ts), n)
        xs = [mp.cos(t) for t in ts]  # ascending t
        # classical Gauss-Jacobi weight:  Gamma ratio * 2^(a+b+1) / ((1-x^2) P_n'(x)^2),
        # with P_n' = (n+a+b+1)/2 * P_{n-1}^(a+1,b+1)
        cst = (mp.gamma(n + a_ + 1) * mp.gamma(n + b_ + 1)
               / (mp.gamma(n + a_ + b_ + 1) * mp.factorial(n)) * mp.power(2, a_ + b_ + 1))

        def dpn(x):
            if n == 0:
                return mp.mpf(0)
            return (n + a_ + b_ + 1) / 2 * jac(n - 1, a_ + 1, b_ + 1, x)

        ws = [cst / ((1 - x * x) * dpn(x) ** 2) for x in xs]

        def hk(k):
            if k == 0:
                return mp.power(2, a_ + b_ + 1) * mp.gamma(a_ + 1) * mp.gamma(b_ + 1) / mp.gamma(a_ + b_ + 2)
            return (mp.power(2, a_ + b_ + 1) / (2 * k + a_ + b_ + 1)
                    * mp.gamma(k + a_ + 1) * mp.gamma(k + b_ + 1)
                    / (mp.gamma(k + a_ + b_ + 1) * mp.factorial(k)))

        norms = [mp.sqrt(hk(k)) for k in range(n)]
        A = np.empty((n, n))
        for j, x in enumerate(xs):
            sw = mp.sqrt(ws[j])
            for k in range(n):
                A[j, k] = float(sw * jac(k, a_, b_, x) / norms[k])
        return A, np.array([float(x) for x in xs]), np.array([float(w) for w in ws])


BRUTE_PAIRS = [(0.0, 0.0), (0.25, -0.35), (-0.4, 0.1), (0.3, 0.3), (0.3, -0.3),
               (-0.5, -0.5), (0.9, -0.9), (-0.75, 0.6)]


@pytest.mark.parametrize("a,b", BRUTE_PAIRS)
@pytest.mark.parametrize("n", [1, 5, 16])
def test_brute_force_mpmath(orc, n, a, b):
    A_ref, x_ref, w_ref = _mp_matrix(n, a, b)
    A, x, w = orc.matrix(n, a, b)
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=2e-16 * 4)
    np.testing.assert_allclose(w, w_ref, rtol=1e-14, atol=0)
    assert np.abs(A - A_ref).max() <= 1e-14
    # and the transform of a random vector
    al = np.random.default_rng(n).standard_normal(n)
    assert np.abs(A @ al - A_ref @ al).max() <= 1e-14 * max(1.0, np.abs(A_ref @ al).max())


@pytest.mark.slow
def test_brute_force_mpmath_legendre_n48(orc):
    A_ref, _, _ = _mp_matrix(48, 0.0, 0.0, dps=30)
    A, _, _ = orc.matrix(48, 0.0, 0.0)
    assert np.abs(A - A_ref).max() <= 1e-14


# ------------------------------------------------------------ quadrature exactness
@pytest.mark.parametrize("a,b", [(0.25, -0.35), (-0.4, 0.1), (0.3, 0.3), (0.7, -0.2), (-0.9, 0.45)])
def test_quadrature_exact_to_degree_2n_minus_1(orc, a, b):
    n = 12
    _, x, w = orc.matrix(n, a, b)
    for k in range(2 * n):
        f = lambda s, k=k: math.cos(k * math.acos(max(-1.0, min(1.0, s))))
        # QAWS: integral of (s+1)^b (1-s)^a f(s) over [-1, 1]
        ref, err = integrate.quad(f, -1.0, 1.0, weight="alg", wvar=(b, a), limit=200,
                                  epsabs=1e-14, epsrel=1e-13)
        got = float(np.sum(w * np.cos(k * np.arccos(x))))
        assert abs(got - ref) <= 2e-13 * max(1.0, abs(ref)), (k, got, ref)


# ------------------------------------------------------------ orthogonality at size
@pytest.mark.parametrize("n,a,b", [(1024, 0.25, -0.35), (1024, -0.4, 0.1), (256, 0.3, 0.3)])
def test_orthogonal_at_benchmark_sizes(orc, n, a, b):
    A, _, _ = orc.matrix(n, a, b)
    assert np.linalg.norm(A.T @ A - np.eye(n), 2) <= 1e-13
    al = np.random.default_rng(7).standard_normal(n)
    rt = A.T @ (A @ al)
    assert np.linalg.norm(rt - al) / np.linalg.norm(al) <= 1e-14


def test_forward_inverse_identity_2d(orc):
    params = ((0.25, -0.35), (-0.4, 0.1))
    al = np.random.default_rng(3).standard_normal((64, 48))
    g = orc.forward(al, params)
    back = orc.inverse(g, params)
    assert np.linalg.norm(back - al) / np.linalg.norm(al) <= 1e-14
    assert abs(np.linalg.norm(g) - np.linalg.norm(al)) <= 1e-13 * np.linalg.norm(al)


# ------------------------------------------------------------ Kronecker convention
def test_kronecker_axis_convention_2d(orc):
    params = ((0.25, -0.35), (-0.4, 0.1))
    n0, n1 = 5, 7
    al = np.random.default_rng(4).standard_normal((n0, n1))
    A0 = orc.matrix(n0, *params[0])[0]
    A1 = orc.matrix(n1, *params[1])[0]
    ref = (np.kron(A0, A1) @ al.reshape(-1)).reshape(n0, n1)
    np.testing.assert_allclose(orc.forward(al, params), ref, rtol=0, atol=1e-14)
    ref_inv = (np.kron(A0, A1).T @ al.reshape(-1)).reshape(n0, n1)
    np.testing.assert_allclose(orc.inverse(al, params), ref_inv, rtol=0, atol=1e-14)


def test_kronecker_axis_convention_3d(orc):
    params = ((0.1, 0.2), (-0.3, 0.4), (0.45, -0.15))
    shape = (3, 4, 5)
    al = np.random.default_rng(5).standard_normal(shape)
    K = np.kron(np.kron(orc.matrix(3, *params[0])[0], orc.matrix(4, *params[1])[0]),
                orc.matrix(5, *params[2])[0])
    np.testing.assert_allclose(orc.forward(al, params), (K @ al.reshape(-1)).reshape(shape),
                               rtol=0, atol=1e-14)


def test_sampled_entries_match_full(orc):
    params = ((0.3, 0.3),) * 3
    al = np.random.default_rng(6).standard_normal((9, 10, 11))
    g = orc.forward(al, params)
    idx = np.array([[0, 0, 0], [8, 9, 10], [4, 2, 7]])
    np.testing.assert_allclose(orc.forward_entries(al, params, idx), g[tuple(idx.T)], atol=1e-14)
    a = orc.inverse(g, params)
    np.testing.assert_allclose(orc.inverse_entries(g, params, idx), a[tuple(idx.T)], atol=1e-14)


# ------------------------------------------------------------ planted mistakes
def test_pins_catch_swapped_parameters(orc):
    """An oracle that swapped a and b (the endpoint convention) fails brute force."""
    A_ref, _, _ = _mp_matrix(8, 0.25, -0.35)
    A_bad, _, _ = orc.matrix(8, -0.35, 0.25)
    assert np.abs(A_bad - A_ref).max() > 1e-3


def test_pins_catch_reversed_node_order(orc):
    A, _, _ = orc.matrix(16, -0.5, -0.5)
    al = np.random.default_rng(8).standard_normal(16)
    ref = scipy.fft.dct(al, type=3, norm="ortho")
    assert np.abs(A[::-1] @ al - ref).max() > 1e-3


def test_rejects_invalid_parameters(orc):
    with pytest.raises(ValueError):
        orc.matrix(8, -1.0, 0.0)
    with pytest.raises(ValueError):
        orc.matrix(0, 0.0, 0.0)


# ------------------------------------------------- modified Jacobi functions (nonuniform)
# Closed forms of Ptilde_k(t) = phat_k(cos t) sqrt(w(cos t) sin t) at the four
# Chebyshev parameter pairs (first to fourth kind): each normalised on (0, pi)
# and positive at t -> 0+ where the polynomial is positive at x = 1.
_PTILDE_CLOSED = {
    (-0.5, -0.5): lambda k, t: np.where(k == 0, np.sqrt(1 / np.pi), np.sqrt(2 / np.pi) * np.cos(k * t)),
    (0.5, 0.5): lambda k, t: np.sqrt(2 / np.pi) * np.sin((k + 1) * t),
    (-0.5, 0.5): lambda k, t: np.sqrt(2 / np.pi) * np.cos((k + 0.5) * t),
    (0.5, -0.5): lambda k, t: np.sqrt(2 / np.pi) * np.sin((k + 0.5) * t),
}


@pytest.mark.parametrize("ab", list(_PTILDE_CLOSED))
def test_ptilde_chebyshev_closed_forms(orc, ab):
    n = 300
    t = np.sort(np.random.default_rng(21).uniform(1e-3, np.pi - 1e-3, 97))
    P = orc.ptilde(n, ab[0], ab[1], t)
    k = np.arange(n)[None, :]
    ref = _PTILDE_CLOSED[ab](k, t[:, None])
    assert np.abs(P - ref).max() <= 1e-13


def test_ptilde_swapped_parameters_fail_the_pin(orc):
    """Planted mistake: (a, b) swapped in the call gives the other kind."""
    t = np.linspace(0.1, 3.0, 11)
    P = orc.ptilde(20, 0.5, -0.5, t)
    ref = _PTILDE_CLOSED[(-0.5, 0.5)](np.arange(20)[None, :], t[:, None])
    assert np.abs(P - ref).max() > 0.1


@pytest.mark.parametrize("a,b", [(0.25, -0.35), (-0.8, 0.6), (0.9, 0.3)])
def test_ptilde_mpmath_definition(orc, a, b):
    """The paper's definition of the modified Jacobi function of the first
    kind (Section 1): C_k P_k^(a,b)(cos t) sin(t/2)^(a+1/2) cos(t/2)^(b+1/2)
    with C_k = sqrt((2k+a+b+1) Gamma(1+k) Gamma(1+k+a+b) / (Gamma(1+k+a) Gamma(1+k+b))),
    P_k from mpmath's own Jacobi function, at 30 digits."""
    n = 14
    t = [0.05, 0.7, 1.5, 2.2, 3.1]
    P = orc.ptilde(n, a, b, np.array(t))
    with mp.workdps(30):
        for j, tj in enumerate(t):
            for k in range(n):
                c = mp.sqrt((2 * k + a + b + 1) * mp.gamma(1 + k) * mp.gamma(1 + k + a + b)
                            / (mp.gamma(1 + k + a) * mp.gamma(1 + k + b)))
                ref = c * mp.jacobi(k, a, b, mp.cos(tj)) * mp.sin(mp.mpf(tj) / 2) ** (a + 0.5) \
                    * mp.cos(mp.mpf(tj) / 2) ** (b + 0.5)
                assert abs(P[j, k] - float(ref)) <= 1e-13 * max(1.0, abs(float(ref))), (j, k)


def test_ptilde_at_gauss_jacobi_nodes_weighted_is_the_uniform_matrix(orc):
    """sqrt(w_j) Ptilde_k(t_j) with the trigonometric weights of eq. (9) is the
    uniform matrix W J (the uniform transform is the nonuniform one at the
    quadrature nodes, with the weights applied)."""
    n, a, b = 200, 0.3, -0.45
    A, x, om = orc.matrix(n, a, b)
    t = np.arccos(x)
    w_trig = om / ((1 - x) ** a * (1 + x) ** b * np.sin(t))
    P = orc.ptilde(n, a, b, t)
    assert np.abs(np.sqrt(w_trig)[:, None] * P - A).max() <= 1e-12


def test_forward_points_kronecker_convention(orc):
    """2D nonuniform forward: f[i, j] = sum_{k,l} alpha[k, l] Ptilde_k(s_i) Ptilde_l(t_j)."""
    rng = np.random.default_rng(5)
    al = rng.standard_normal((7, 9))
    s, t = rng.uniform(0.1, 3.0, 7), rng.uniform(0.1, 3.0, 9)
    ab = ((0.2, -0.1), (-0.3, 0.4))
    P0, P1 = orc.ptilde(7, *ab[0], s), orc.ptilde(9, *ab[1], t)
    ref = np.kron(P0, P1) @ al.ravel()
    assert np.abs(orc.forward_points(al, ab, (s, t)).ravel() - ref).max() <= 1e-13


# ------------------------------------------------- plain fp64 path (long 1D items)
@pytest.mark.parametrize("n", [1, 5, 64, 65, 4096])
def test_fp64_path_chebyshev_closed_forms(orc, n):
    """Nodes and transforms at a = b = -1/2 (DCT-III / DCT-II) and a = b = 1/2
    (DST-I).  The bound grows like n^2 * 4e-16: the nodes next to x = +-1 are
    held in fp64 x, and phat_k for k ~ n turns an error of one unit in the
    last place of x into about n^2 * 1e-16 there (a limit of the fp64 path,
    far below the fp32-bulk bar it serves)."""
    tol = max(1e-12, 4e-16 * n * n)
    j = np.arange(1, n + 1)
    x, w = orc.nodes_fp64(n, -0.5, -0.5)
    np.testing.assert_allclose(x, np.cos((2 * j - 1) * np.pi / (2 * n)), rtol=0, atol=4e-15)
    v = np.random.default_rng(n).standard_normal(n)
    ref = scipy.fft.dct(v, type=3, norm="ortho")
    assert np.abs(orc.apply1d_fp64(v, (-0.5, -0.5)) - ref).max() <= tol * max(1.0, np.abs(ref).max())
    assert np.abs(orc.apply1d_fp64(v, (-0.5, -0.5), True) - scipy.fft.dct(v, type=2, norm="ortho")).max() <= tol
    x, w = orc.nodes_fp64(n, 0.5, 0.5)
    np.testing.assert_allclose(x, np.cos(j * np.pi / (n + 1)), rtol=0, atol=4e-15)
    assert np.abs(orc.apply1d_fp64(v, (0.5, 0.5)) - scipy.fft.dst(v, type=1, norm="ortho")).max() <= tol


@pytest.mark.parametrize("n,a,b", [(64, 0.25, -0.35), (1000, -0.9, 0.8), (4096, 0.4, 0.1)])
def test_fp64_path_matches_long_double_build(orc, n, a, b):
    """Against the long-double construction (itself pinned above): nodes and the
    transform in both directions."""
    A, x, om = orc.matrix(n, a, b)
    xf, wf = orc.nodes_fp64(n, a, b)
    assert np.abs(xf - x).max() <= 1e-14
    v = np.random.default_rng(3).standard_normal(n)
    assert np.linalg.norm(orc.apply1d_fp64(v, (a, b)) - A @ v) <= 1e-10 * np.linalg.norm(v)
    assert np.linalg.norm(orc.apply1d_fp64(v, (a, b), True) - A.T @ v) <= 1e-10 * np.linalg.norm(v)


def test_fp64_path_orthogonal_at_the_largest_size(orc):
    """At n = 16384 (the longest 1D item): the map is orthogonal, so the
    round trip returns v and the norm is kept."""
    n, ab = 16384, (-0.35, 0.45)
    v = np.random.default_rng(4).standard_normal(n)
    g = orc.apply1d_fp64(v, ab)
    assert abs(np.linalg.norm(g) / np.linalg.norm(v) - 1) <= 1e-10
    assert np.linalg.norm(orc.apply1d_fp64(g, ab, True) - v) <= 1e-9 * np.linalg.norm(v)


# ------------------------------------------------- second kind (Qtilde)
# Chebyshev cases: with Ptilde_k + i Qtilde_k = M exp(i psi) and psi
# increasing, the four Chebyshev kinds give Qtilde as the matching sine or
# cosine (the finite Hilbert transforms of T_k, U_k, V_k and W_k with their
# weights are multiples of U_{k-1}, T_{k+1}, W_k and V_k).
_QTILDE_CLOSED = {
    (-0.5, -0.5): lambda k, t: np.where(k == 0, 0.0, np.sqrt(2 / np.pi) * np.sin(k * t)),
    (0.5, 0.5): lambda k, t: -np.sqrt(2 / np.pi) * np.cos((k + 1) * t),
    (-0.5, 0.5): lambda k, t: np.sqrt(2 / np.pi) * np.sin((k + 0.5) * t),
    (0.5, -0.5): lambda k, t: -np.sqrt(2 / np.pi) * np.cos((k + 0.5) * t),
}


@pytest.mark.parametrize("ab", list(_QTILDE_CLOSED))
def test_qtilde_chebyshev_closed_forms(orc, ab):
    n = 300
    t = np.sort(np.random.default_rng(22).uniform(1e-3, np.pi - 1e-3, 97))
    Q = orc.qtilde(n, ab[0], ab[1], t)
    ref = _QTILDE_CLOSED[ab](np.arange(n)[None, :], t[:, None])
    assert np.abs(Q - ref).max() <= 1e-12


def test_uniform_second_kind_matrix_chebyshev(orc):
    """a = b = -1/2: nodes (2j-1) pi / 2n, trigonometric weights pi / n, so the
    matrix is sqrt(2/n) sin(k t_j) (k >= 1) with a zero first column."""
    n = 64
    Q = orc.matrix_q(n, -0.5, -0.5)
    t = (2 * np.arange(1, n + 1) - 1) * np.pi / (2 * n)
    k = np.arange(n)[None, :]
    ref = np.where(k == 0, 0.0, np.sqrt(2.0 / n) * np.sin(k * t[:, None]))
    assert np.abs(Q - ref).max() <= 1e-13


def _q_mpmath(k, a, b, x):
    """q_k(x) = PV int w(s) phat_k(s) / (s - x) ds at 30 digits: the principal
    value written as a regular integral plus w(x) phat_k(x) log((1-x)/(1+x)),
    each half mapped so that the endpoint power singularity goes away
    (s = 1 - (1-x) v^p with p = 1/(1+a) on the right, likewise on the left)."""
    with mp.workdps(30):
        a, b, x = mp.mpf(a), mp.mpf(b), mp.mpf(x)
        hk = (2 ** (a + b + 1) / (2 * k + a + b + 1) * mp.gamma(k + a + 1) * mp.gamma(k + b + 1)
              / (mp.gamma(k + a + b + 1) * mp.factorial(k)))
        ph = lambda s: mp.jacobi(k, a, b, s) / mp.sqrt(hk)  # noqa: E731
        wx = (1 - x) ** a * (1 + x) ** b
        fx = wx * ph(x)
        pa, pb = max(mp.mpf(1), 1 / (1 + a)), max(mp.mpf(1), 1 / (1 + b))

        def right(v):
            s = 1 - (1 - x) * v ** pa
            ws = (1 - x) ** a * v ** (pa * (1 + a) - 1) * (1 + s) ** b * ph(s)
            return (ws - fx * v ** (pa - 1)) / (s - x) * (1 - x) * pa

        def left(v):
            s = -1 + (1 + x) * v ** pb
            ws = (1 + x) ** b * v ** (pb * (1 + b) - 1) * (1 - s) ** a * ph(s)
            return (ws - fx * v ** (pb - 1)) / (s - x) * (1 + x) * pb

        return mp.quad(left, [0, 1]) + mp.quad(right, [0, 1]) + fx * mp.log((1 - x) / (1 + x))


@pytest.mark.parametrize("a,b", [(0.25, -0.35), (-0.8, 0.6), (0.9, 0.3), (-0.95, -0.9)])
def test_qtilde_against_principal_value_quadrature(orc, a, b):
    """Independent of the oracle's closed form for q_0 and of its recurrence:
    every q_k (k < 8) from its own principal-value integral."""
    xs = [-0.99, -0.7, 0.2, 0.95]
    t = np.arccos(xs)
    Q = orc.qtilde(8, a, b, t)
    for j, x in enumerate(xs):
        w = (1 - x) ** a * (1 + x) ** b
        for k in range(8):
            ref = float(mp.sqrt(mp.sin(t[j]) / w) * _q_mpmath(k, a, b, x) / mp.pi)
            assert abs(Q[j, k] - ref) <= 1e-13 * max(1.0, abs(ref)), (x, k, Q[j, k], ref)


def test_first_and_second_kind_share_a_non_oscillatory_amplitude(orc):
    """Ptilde_k^2 + Qtilde_k^2 = M^2 varies slowly and tends to 2/pi at high
    degree away from the endpoints (a dropped 1/pi or a wrong power of
    w(x) / sin t in Qtilde breaks this)."""
    t = np.linspace(0.4, np.pi - 0.4, 50)
    for a, b in ((0.25, -0.35), (-0.4, 0.1), (0.45, 0.45)):
        P, Q = orc.ptilde(401, a, b, t), orc.qtilde(401, a, b, t)
        m2 = P[:, 400] ** 2 + Q[:, 400] ** 2
        assert np.abs(m2 - 2 / np.pi).max() <= 2e-3
        # smooth in t: no oscillation at the degree's frequency
        assert np.abs(np.diff(m2, 2)).max() <= 1e-4


def test_qtilde_swapped_parameters_fail_the_pin(orc):
    t = np.linspace(0.1, 3.0, 11)
    Q = orc.qtilde(20, 0.5, -0.5, t)
    ref = _QTILDE_CLOSED[(-0.5, 0.5)](np.arange(20)[None, :], t[:, None])
    assert np.abs(Q - ref).max() > 0.1


def test_uniform_second_kind_is_the_weighted_nonuniform_one(orc):
    n, a, b = 200, 0.3, -0.45
    A, x, om = orc.matrix(n, a, b)
    t = np.arccos(x)
    w_trig = om / ((1 - x) ** a * (1 + x) ** b * np.sin(t))
    assert np.abs(np.sqrt(w_trig)[:, None] * orc.qtilde(n, a, b, t) - orc.matrix_q(n, a, b)).max() <= 1e-11


def test_second_kind_refuses_parameters_the_closed_form_lacks(orc):
    with pytest.raises(ValueError):
        orc.qtilde(10, 0.0, 0.3, [1.0])
    assert np.all(np.isfinite(orc.qtilde(10, 0.0, 0.0, [0.5, 1.0])))


def test_qtilde_legendre_against_scipy(orc):
    """a = b = 0: q_k = PV int phat_k(s) / (s - x) ds = -2 sqrt(k + 1/2) Q_k(x)
    with Q_k the Legendre function of the second kind (Neumann's integral),
    from scipy.special.lqn."""
    from scipy.special import lqn

    xs = np.array([-0.9, -0.3, 0.1, 0.6, 0.97])
    Q = orc.qtilde(30, 0.0, 0.0, np.arccos(xs))
    for j, x in enumerate(xs):
        ql, _ = lqn(29, x)
        ref = np.sqrt(np.sin(np.arccos(x))) * (-2 * np.sqrt(np.arange(30) + 0.5) * ql) / np.pi
        assert np.abs(Q[j] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
