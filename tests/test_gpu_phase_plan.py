"""GPU parity of transforms planned by the phase functions (Section 2.2):
nodes, weights and sampled columns of Algorithm 2.1 from the nonoscillatory
phase and amplitude tables (planner 2), applied by the HIP path through the C
ABI, against the oracle.

1D at 1024 to 16384 points (the 4096-item batch's range) and 2D at
1024 x 1024 (the automatic planner picks the tables there), forward and
inverse.  The oracle side is its plain fp64 path (apply1d_fp64: safeguarded
Newton nodes, recurrence sums) for 1D and its dense matrices for 2D.
Bars: rel-l2 <= 5 tol per axis on the fp64 path (the factorization error is
at most tol per axis; the tables add about 1e-9 at 16384 points), 2e-5 on the
fp32-bulk path at tol 1e-7.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def jt():
    import paper_1901_07275_amd as m

    return m


def relerr(x, ref):
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


def run(plan, x, prec, direction):
    dev = _dev()
    t = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    out = plan.forward(t, prec=prec) if direction == 0 else plan.inverse(t, prec=prec)
    torch.cuda.synchronize()
    return out.cpu().numpy()


CASES_1D = [(n, a, b, prec) for n, a, b in [(1024, 0.25, -0.35), (4096, -0.45, 0.4)] for prec in (0, 1)]
CASES_1D += [(8192, 0.1, -0.2, 0), (16384, 0.3, 0.3, 1)]  # the fp64 path's longest line is 8192


@pytest.mark.parametrize("n,a,b,prec", CASES_1D)
def test_phase_planned_1d(jt, orc, n, a, b, prec):
    tol, bar = (1e-8, 5e-8) if prec == 0 else (1e-7, 2e-5)
    print("phase plan 1D n=%d a=%g b=%g prec=%d" % (n, a, b, prec), flush=True)
    plan = jt.Plan((n,), ((a, b),), tol, planner=2).bind(_dev())
    assert plan.info(0)["planner"] == 2
    rng = np.random.default_rng(n + prec)
    al = rng.standard_normal(n)
    g = run(plan, al, prec, 0)
    ef = relerr(g, orc.apply1d_fp64(al, (a, b)))
    gi = rng.standard_normal(n)
    back = run(plan, gi, prec, 1)
    ei = relerr(back, orc.apply1d_fp64(gi, (a, b), transpose=True))
    print("  forward rel-l2 %.3e inverse rel-l2 %.3e (rank %d)" % (ef, ei, plan.info(0)["rank"]))
    assert ef <= bar and ei <= bar


def test_phase_planned_2d(jt, orc):
    ab = ((0.25, -0.35), (-0.4, 0.1))
    tol = 1e-8
    print("phase plan 2D 1024 x 1024", flush=True)
    plan = jt.Plan((1024, 1024), ab, tol).bind(_dev())
    assert plan.info(0)["planner"] == 2 and plan.info(1)["planner"] == 2
    al = np.random.default_rng(77).standard_normal((1024, 1024))
    g = run(plan, al, 0, 0)
    ref = orc.forward(al, ab)
    ef = relerr(g, ref)
    back = run(plan, ref, 0, 1)
    ei = relerr(back, al)
    print("  forward rel-l2 %.3e round trip via the oracle's g %.3e" % (ef, ei))
    assert ef <= 2 * 5 * tol and ei <= 2 * 5 * tol
