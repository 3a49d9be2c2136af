"""Planning by the nonoscillatory phase and amplitude functions (Section 2.2,
eqs. (phase:Neq), (phase:mpsip), (cheby:bary); Algorithm 2.1 of Section 2.1 on
O(r) sampled rows and columns), checked on the host against the oracle:

* the nodes solve psi = pi/2 (mod pi) and the weights are pi / psi': both
  against the oracle's long double Gauss-Jacobi rule;
* the sampled columns come from the tables: the plan's factors U V^T must
  reproduce the oracle's W B = (A + i Q) o exp(-2 pi i m_j k / L) (A, Q the
  oracle's first- and second-kind matrices at the plan's bins m_j) to the
  plan's tolerance, and the r-FFT formulas of eqs. (50), (51) applied to the
  factors must reproduce A alpha and A^T g;
* planner 2 and planner 1 reach the same ranks.
Runs through the C ABI only (no GPU)."""
import numpy as np
import pytest

import paper_1901_07275_amd as jt
from test_plan import _emulated_forward, _emulated_inverse


def plan1(n, a, b, tol, **kw):
    return jt.Plan([n], [(a, b)], tol, **kw)


@pytest.mark.parametrize("n,a,b,tol,planner,kind,expect", [
    (1024, 0.25, -0.35, 1e-7, 0, 1, 2),    # automatic from 1024 points
    (1023, 0.25, -0.35, 1e-7, 0, 1, 1),    # below the automatic crossover
    (200, 0.25, -0.35, 1e-7, 2, 1, 2),     # forced
    (2048, 0.25, -0.35, 1e-9, 0, 1, 1),    # tolerance below 1e-8
    (2048, 0.25, -0.35, 1e-9, 2, 1, 1),
    (2048, 0.6, -0.35, 1e-7, 2, 1, 1),     # outside (-1/2, 1/2)
    (2048, 0.25, -0.5, 1e-7, 2, 1, 1),
    (2048, 0.25, -0.35, 1e-7, 1, 1, 1),    # recurrence requested
    (2048, 0.25, -0.35, 1e-7, 0, 2, 2),    # second kind
])
def test_phase_planner_is_used_where_it_applies(n, a, b, tol, planner, kind, expect):
    P = plan1(n, a, b, tol, planner=planner, kind=kind)
    assert P.info(0)["planner"] == expect


def test_planner_option_is_checked():
    with pytest.raises(RuntimeError):
        plan1(256, 0.1, 0.1, 1e-7, planner=3)


def test_points_plans_use_the_recurrence():
    t = np.sort(np.random.default_rng(3).uniform(0.1, 3.0, 1500))
    P = jt.Plan.at_points([t], [(0.1, 0.2)], 1e-7)
    assert P.info(0)["planner"] == 1


@pytest.mark.parametrize("n", [64, 333, 2048])
@pytest.mark.parametrize("a,b", [(0.49, -0.49), (-0.3, 0.2), (0.0, 0.0), (-0.45, -0.45)])
def test_phase_nodes_and_weights_match_oracle(orc, n, a, b):
    _, xo, wo = orc.matrix(n, a, b)
    P = plan1(n, a, b, 1e-8, planner=2)
    assert P.info(0)["planner"] == 2
    t, x, w = P.nodes(0)
    assert np.all(np.diff(t) > 0)
    np.testing.assert_allclose(x, xo, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, wo, rtol=3e-12, atol=0)


def _oracle_wb(orc, P, n, a, b):
    """W B of eq. (45) from the oracle's matrices, with the plan's bins."""
    bins, _, _, _ = P.factors(0)
    inf = P.info(0)
    L, nu0 = inf["L"], inf["nu0"]
    A = orc.matrix(n, a, b)[0]
    Q = orc.matrix_q(n, a, b)
    k = np.arange(nu0, n)
    ph = np.exp(-2j * np.pi * ((np.outer(bins.astype(np.int64), k) % L) / L))
    return (A[:, nu0:] + 1j * Q[:, nu0:]) * ph


@pytest.mark.parametrize("n,a,b,tol", [(1500, 0.25, -0.35, 1e-8), (2048, -0.45, 0.45, 1e-7),
                                       (700, 0.1, 0.2, 1e-8), (1024, 0.0, 0.0, 1e-7)])
def test_phase_plan_factors_reproduce_oracle(orc, n, a, b, tol):
    P = plan1(n, a, b, tol, planner=2)
    inf = P.info(0)
    assert inf["planner"] == 2 and inf["rel_err"] <= tol
    _, _, U, V = P.factors(0)
    WB = _oracle_wb(orc, P, n, a, b)
    err = np.linalg.norm(U.T @ V - WB) / np.linalg.norm(WB)
    assert err <= 2 * tol, err
    # the r-FFT forms of eqs. (50), (51) on these factors
    A = orc.matrix(n, a, b)[0]
    al = np.random.default_rng(n + 5).standard_normal(n)
    g = _emulated_forward(P, 0, al)
    assert np.linalg.norm(g - A @ al) / np.linalg.norm(A @ al) <= 3 * tol
    back = _emulated_inverse(P, 0, A @ al)
    assert np.linalg.norm(back - al) / np.linalg.norm(al) <= 3 * tol
    # the same rank as the recurrence planner (both meet tol on the same matrix)
    assert abs(plan1(n, a, b, tol, planner=1).info(0)["rank"] - inf["rank"]) <= 1


def test_phase_plan_second_kind(orc):
    """Second kind: the factors hold -i W B (Im(u y) = Re((-i u) y))."""
    n, a, b, tol = 1200, 0.3, -0.2, 1e-8
    P = plan1(n, a, b, tol, planner=2, kind=2)
    assert P.info(0)["planner"] == 2
    _, wv, U, V = P.factors(0)
    WB = _oracle_wb(orc, P, n, a, b)
    err = np.linalg.norm(U.T @ V - (-1j) * WB) / np.linalg.norm(WB)
    assert err <= 2 * tol, err
    Q = orc.matrix_q(n, a, b)
    nu0 = P.info(0)["nu0"]
    np.testing.assert_allclose(wv, Q[:, :nu0].T, rtol=0, atol=1e-13 * np.abs(Q).max())


def test_phase_plan_is_deterministic():
    p1 = plan1(3000, 0.2, 0.1, 1e-7, planner=2)
    p2 = plan1(3000, 0.2, 0.1, 1e-7, planner=2)
    for x, y in zip(p1.factors(0), p2.factors(0)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("a,b", [(0.2, -0.1), (0.45, -0.45), (-0.3, 0.3)])
@pytest.mark.parametrize("k", [27, 100, 1000])
def test_wronskian_of_the_normalized_pair(orc, a, b, k):
    """The tables take psi' = W / N with W = 2 lam / pi, lam = k + (a+b+1)/2,
    for the pair (Ptilde_k, Qtilde_k) as the oracle defines it: checked here on
    the oracle alone, W = P Q' - P' Q from central differences at several t."""
    lam = k + (a + b + 1) / 2
    t = np.array([0.4, 1.1, np.pi / 2, 2.3, 2.9])
    h = 1e-5
    tt = np.concatenate([t - h, t, t + h])
    P = orc.ptilde(k + 1, a, b, tt)[:, k].reshape(3, -1)
    Q = orc.qtilde(k + 1, a, b, tt)[:, k].reshape(3, -1)
    dP = (P[2] - P[0]) / (2 * h)
    dQ = (Q[2] - Q[0]) / (2 * h)
    W = P[1] * dQ - dP * Q[1]
    # central differences: error ~ h^2 lam^3 relative to lam
    np.testing.assert_allclose(W, 2 * lam / np.pi, rtol=max(1e-6, 2 * h * h * lam ** 2))


def test_phase_nodes_follow_the_amplitude(orc):
    """At a zero of Ptilde_n the weight pi / psi' equals pi N / W; with W = 2 lam / pi
    and N = Ptilde^2 + Qtilde^2 = Qtilde^2 there, the Gauss weights in t are
    pi^2 Qtilde_n(t_j)^2 / (2 lam): checked on the oracle's own rule."""
    n, a, b = 300, 0.3, -0.2
    _, x, w = orc.matrix(n, a, b)
    t = np.arccos(x)
    Q = orc.qtilde(n + 1, a, b, t)[:, n]
    lam = n + (a + b + 1) / 2
    wt = w / ((1 - x) ** a * (1 + x) ** b * np.sin(t))
    np.testing.assert_allclose(wt, np.pi ** 2 * Q ** 2 / (2 * lam), rtol=1e-9)
