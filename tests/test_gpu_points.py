"""GPU parity of the nonuniform forward transform (jt_plan_points): the HIP
path through the C ABI against the oracle's dense evaluation of
f = (P0 (x) P1 (x) ...) alpha with P_i[j, k] = Ptilde_k(t_{i,j}) (Section 3.1,
the nonuniform remark after eq. (39); Sections 3.2-3.3 for 2D and 3D).

Points: sorted i.i.d. uniform in (0, pi) (the paper's nonuniform experiments
use points other than the quadrature nodes and do not say which), plus a
clustered set (half the points inside an interval of width 1e-3, so hundreds
share one DFT bin) and a set crowding both endpoints.  Bars as for the
uniform transform: rel-l2 <= 1e-11 for fp64 at tol 1e-12, 2e-5 for fp32 bulk
at tol 1e-7.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BAR = {0: (1e-12, 1e-11), 1: (1e-7, 2e-5)}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def jt():
    import paper_1901_07275_amd as m

    return m


def points(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return np.sort(rng.uniform(0.0, np.pi, n))
    if kind == "clustered":
        return np.sort(np.concatenate([rng.uniform(1.0, 1.0 + 1e-3, n // 2), rng.uniform(0.0, np.pi, n - n // 2)]))
    return np.sort(np.concatenate([rng.uniform(1e-6, 1e-3, n // 4), rng.uniform(np.pi - 1e-3, np.pi - 1e-6, n // 4),
                                   rng.uniform(0.0, np.pi, n - 2 * (n // 4))]))


def relerr(x, ref):
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


def forward(jt, plan, al, prec, tin=None):
    dev = _dev()
    x = torch.from_numpy(np.ascontiguousarray(al)).to(dev, tin or torch.float64)
    out = torch.empty(plan.n, dtype=torch.float64, device=dev)
    plan.forward(x, out, prec=prec)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n", [1, 17, 64, 100, 300, 1024, 2047, 4096])
@pytest.mark.parametrize("prec", [0, 1])
def test_points_1d_sizes(jt, orc, n, prec):
    tol, bar = BAR[prec]
    ab = ((0.25, -0.35),)
    t = points("uniform", n, n)
    plan = jt.Plan.at_points([t], ab, tol).bind(_dev())
    al = np.random.default_rng(n + 1).standard_normal(n)
    e = relerr(forward(jt, plan, al, prec), orc.forward_points(al, ab, [t]))
    assert e <= bar, (n, prec, e)


@pytest.mark.parametrize("kind", ["clustered", "ends"])
@pytest.mark.parametrize("prec", [0, 1])
def test_points_1d_clustered_and_endpoints(jt, orc, kind, prec):
    tol, bar = BAR[prec]
    n, ab = 1500, ((-0.3, 0.2),)
    t = points(kind, n, 5)
    plan = jt.Plan.at_points([t], ab, tol).bind(_dev())
    al = np.random.default_rng(6).standard_normal(n)
    e = relerr(forward(jt, plan, al, prec), orc.forward_points(al, ab, [t]))
    assert e <= bar, (kind, prec, e)


@pytest.mark.parametrize("shape,prec", [((200, 300), 0), ((300, 200), 1), ((1024, 1024), 0), ((1024, 1024), 1),
                                        ((33, 1000), 0)])
def test_points_2d(jt, orc, shape, prec):
    tol, bar = BAR[prec]
    ab = ((0.4, 0.4), (0.4, 0.4)) if shape[0] == 1024 else ((0.25, -0.35), (-0.4, 0.1))
    pts = [points("uniform", n, 10 + i) for i, n in enumerate(shape)]
    plan = jt.Plan.at_points(pts, ab, tol).bind(_dev())
    al = np.random.default_rng(sum(shape)).standard_normal(shape)
    e = relerr(forward(jt, plan, al, prec), orc.forward_points(al, ab, pts))
    print("points 2D %s prec %d rel-l2 %.2e" % (shape, prec, e))
    assert e <= bar


@pytest.mark.parametrize("shape,prec", [((64, 65, 66), 0), ((64, 65, 66), 1), ((128, 128, 128), 1)])
def test_points_3d(jt, orc, shape, prec):
    tol, bar = BAR[prec]
    ab = ((0.4, 0.4),) * 3
    pts = [points("uniform", n, 20 + i) for i, n in enumerate(shape)]
    plan = jt.Plan.at_points(pts, ab, tol).bind(_dev())
    al = np.random.default_rng(3).standard_normal(shape)
    e = relerr(forward(jt, plan, al, prec), orc.forward_points(al, ab, pts))
    print("points 3D %s prec %d rel-l2 %.2e" % (shape, prec, e))
    assert e <= bar


def test_points_plan_has_no_inverse(jt):
    t = points("uniform", 200, 1)
    plan = jt.Plan.at_points([t], ((0.1, 0.1),), 1e-8).bind(_dev())
    x = torch.zeros(200, dtype=torch.float64, device=_dev())
    with pytest.raises(jt.JTError) as e:
        plan.inverse(x)
    assert e.value.status == jt.JT_EUNSUPPORTED
    with pytest.raises(jt.JTError) as e:
        jt.Batch([plan], [jt.INVERSE], [0], [0])
    assert e.value.status == jt.JT_EUNSUPPORTED


def test_points_items_in_a_batch(jt, orc):
    """Nonuniform items beside uniform ones in one persistent launch."""
    dev = _dev()
    tp = [points("uniform", 500, 31), points("uniform", 70, 32)]
    P = [jt.Plan.at_points([tp[0]], ((0.2, -0.1),), 1e-7), jt.Plan((300,), ((0.1, 0.1),), 1e-7),
         jt.Plan.at_points([tp[1], tp[0]], ((0.2, -0.1), (0.3, 0.3)), 1e-7)]
    arena = jt.PlanArena(P, dev)
    shapes = [(500,), (300,), (70, 500)]
    sizes = [int(np.prod(s)) for s in shapes]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)
    B = jt.Batch(P, [jt.FORWARD] * 3, offs, offs, jt.F64, jt.F64, jt.PREC_FP32_BULK).bind(dev)
    xs = [np.random.default_rng(i).standard_normal(s) for i, s in enumerate(shapes)]
    inp = torch.from_numpy(np.concatenate([x.ravel() for x in xs])).to(dev)
    out = torch.full_like(inp, float("nan"))
    B.run(inp, out)
    torch.cuda.synchronize()
    assert B.errors() == 0
    o = out.cpu().numpy()
    refs = [orc.forward_points(xs[0], ((0.2, -0.1),), [tp[0]]), orc.forward(xs[1], ((0.1, 0.1),)),
            orc.forward_points(xs[2], ((0.2, -0.1), (0.3, 0.3)), [tp[1], tp[0]])]
    for i in range(3):
        assert relerr(o[offs[i]:offs[i] + sizes[i]].reshape(shapes[i]), refs[i]) <= 2e-5, i
    del arena
