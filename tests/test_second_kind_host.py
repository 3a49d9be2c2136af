"""Host checks of second-kind plans (no GPU): the r scaled FFTs of eq. (50)
evaluated with numpy on the plan's own factors reproduce the oracle's
second-kind transforms, uniform (sqrt(w_j) Qtilde_k(t_j) at the Gauss-Jacobi
nodes) and at given points (Qtilde_k(t_j)); the plan's companion q_0
(quadrature) and the oracle's (Tricomi's closed form) are independent."""
import numpy as np
import pytest

import paper_1901_07275_amd as jt
from test_points_host import fft_formula, points


@pytest.mark.parametrize("n,ab,tol", [(300, (0.25, -0.35), 1e-12), (1000, (-0.4, 0.1), 1e-7),
                                      (700, (0.45, 0.45), 1e-10), (513, (-0.9, 0.8), 1e-12), (40, (0.3, 0.2), 1e-12)])
def test_second_kind_plan_reproduces_the_oracle(orc, n, ab, tol):
    al = np.random.default_rng(n).standard_normal(n)
    p = jt.Plan((n,), (ab,), tol, kind=2)
    ref = orc.forward_q(al, (ab,))
    assert np.linalg.norm(fft_formula(p, 0, al) - ref) <= 3 * tol * np.linalg.norm(ref)
    t = points("uniform", n, n + 1)
    q = jt.Plan.at_points([t], (ab,), tol, kind=2)
    ref = orc.forward_points_q(al, (ab,), [t])
    assert np.linalg.norm(fft_formula(q, 0, al) - ref) <= 3 * tol * np.linalg.norm(ref)


def test_second_kind_shares_the_first_kinds_low_rank_factors():
    """The second kind is the imaginary part of the same W B: its factors are
    the first kind's with u turned by -i, and v unchanged."""
    n, ab, tol = 600, (0.2, -0.3), 1e-10
    b1, wv1, u1, v1 = jt.Plan((n,), (ab,), tol).factors(0)
    b2, wv2, u2, v2 = jt.Plan((n,), (ab,), tol, kind=2).factors(0)
    assert np.array_equal(b1, b2) and np.array_equal(v1, v2)
    assert np.array_equal(u2, -1j * u1)
    assert not np.allclose(wv1, wv2)


def test_kind_is_checked():
    with pytest.raises(jt.JTError) as e:
        jt.Plan((100,), ((0.1, 0.1),), 1e-8, kind=3)
    assert e.value.status == jt.JT_EINVAL
