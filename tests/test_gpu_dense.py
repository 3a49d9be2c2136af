"""GPU parity of the dense matrix-core pass: axes shorter than the plan's
dense_below keep the whole n x n matrix and are applied with MFMA tiles.
There is no low-rank error on such an axis, so fp64 is held to 1e-12 and
fp32 to 2e-5 (plus 20 tol per FFT axis when the other axes use FFTs)."""
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


CASES = [((17,), ((0.1, 0.2),)), ((100,), ((0.3, -0.2),)), ((257,), ((0.0, 0.0),)), ((1024,), ((0.25, -0.35),)),
         ((40, 130), ((0.25, -0.35), (-0.4, 0.1))), ((130, 33), ((0.1, 0.1), (0.2, 0.3))),
         ((5, 20, 37), ((0.1, 0.1), (0.2, 0.3), (0.0, 0.4))), ((300, 700), ((0.2, 0.2), (0.1, -0.3)))]


@pytest.mark.parametrize("shape,ab", CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_dense_pass(jt, orc, shape, ab, prec):
    dev = _dev()
    tol = 1e-12 if prec == 0 else 1e-7
    plan = jt.Plan(shape, ab, tol, dense_below=600).bind(dev)
    dense_axes = [i for i in range(len(shape)) if plan.info(i)["nu0"] == shape[i]]
    assert dense_axes == [i for i in range(len(shape)) if shape[i] < 600]
    al = np.random.default_rng(sum(shape)).standard_normal(shape)
    x = torch.from_numpy(al).to(dev)
    g = plan.forward(x, prec=prec)
    back = g.clone()
    plan.inverse(back, back, prec=prec)  # in place
    torch.cuda.synchronize()
    lim = 1e-11 if prec == 0 else 2e-5
    assert relerr(g.cpu().numpy(), orc.forward(al, ab)) <= lim
    assert relerr(back.cpu().numpy(), al) <= lim


def test_dense_unit_columns_exact(jt, orc):
    """Columns of the dense fp64 matrix equal the oracle's to rounding."""
    dev = _dev()
    n, ab = 200, ((0.25, -0.35),)
    plan = jt.Plan((n,), ab, 1e-12, dense_below=256).bind(dev)
    A = orc.matrix(n, *ab[0])[0]
    for k in (0, 1, 99, 199):
        e = torch.zeros(n, dtype=torch.float64, device=dev)
        e[k] = 1.0
        col = plan.forward(e, prec=0)
        torch.cuda.synchronize()
        assert np.abs(col.cpu().numpy() - A[:, k]).max() <= 1e-13


def test_dense_and_fft_items_in_one_batch(jt, orc):
    dev = _dev()
    shapes = [(100,), (40, 130), (300,), (5, 20, 37), (64, 64), (2000,)]
    abs_ = [((0.1, 0.2),), ((0.25, -0.35), (-0.4, 0.1)), ((0.3, 0.3),), ((0.1, 0.1), (0.2, 0.3), (0.0, 0.4)),
            ((0.1, 0.1), (0.2, 0.2)), ((0.2, 0.1),)]
    dirs = [jt.FORWARD, jt.INVERSE] * 3
    for prec, tol in ((1, 1e-7), (0, 1e-12)):
        plans = jt.plan_many(shapes, abs_, tol, dense_below=[200] * len(shapes))
        arena = jt.PlanArena(plans, dev)
        sizes = [int(np.prod(s)) for s in shapes]
        offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)
        B = jt.Batch(plans, dirs, offs, offs, jt.F64, jt.F64, prec).bind(dev)
        xs = [np.random.default_rng(i).standard_normal(s) for i, s in enumerate(shapes)]
        inp = torch.from_numpy(np.concatenate([x.ravel() for x in xs])).to(dev)
        out = torch.full_like(inp, float("nan"))
        B.run(inp, out)
        torch.cuda.synchronize()
        assert B.errors() == 0
        o = out.cpu().numpy()
        for i, (s, ab) in enumerate(zip(shapes, abs_)):
            ref = orc.forward(xs[i], ab) if dirs[i] == jt.FORWARD else orc.inverse(xs[i], ab)
            got = o[offs[i]:offs[i] + sizes[i]].reshape(s)
            assert relerr(got, ref) <= (1e-11 if prec == 0 else 2e-5), (prec, s)
        del arena
