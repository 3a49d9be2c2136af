"""GPU parity of the batched form: many independent transforms of uneven n,
d and (a, b) in one persistent launch, against the oracle item by item.

Tolerances as in the single-transform tests: fp32-bulk (tol 1e-7) 2e-5
rel-l2, fp64 1e-11 at tol 1e-12, per item in every dimension.  A graph replay must equal the eager run
bit for bit (the arithmetic of a unit does not depend on which block runs it).
"""
import numpy as np
import pytest

import workloads

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


class Prepared:
    """Plans, bound factors, flat input/output buffers and a bound batch."""

    def __init__(self, jt, shapes, abs_, dirs, tol, prec, tin=None, tout=None, seed=0, xs=None, **bopt):
        dev = _dev()
        tin = jt.F64 if tin is None else tin
        tout = jt.F64 if tout is None else tout
        self.shapes, self.abs_, self.dirs = shapes, abs_, dirs
        self.plans = jt.plan_many(shapes, abs_, tol)
        self.arena = jt.PlanArena(self.plans, dev)
        self.sizes = [int(np.prod(s)) for s in shapes]
        self.offs = np.concatenate([[0], np.cumsum(self.sizes)[:-1]]).astype(int)
        self.batch = jt.Batch(self.plans, dirs, self.offs, self.offs, tin, tout, prec, **bopt).bind(dev)
        rng = np.random.default_rng(seed)
        self.xs = xs if xs is not None else [rng.standard_normal(s) for s in shapes]
        tdt = {jt.F64: torch.float64, jt.F32: torch.float32}
        flat = np.concatenate([x.ravel() for x in self.xs])
        self.inp = torch.from_numpy(flat).to(dev, tdt[tin])
        self.out = torch.full((sum(self.sizes),), float("nan"), dtype=tdt[tout], device=dev)
        # what the kernels actually read (after any cast to fp32)
        self.xs_cast = [x.astype(np.float32).astype(np.float64) if tin == jt.F32 else x for x in self.xs]

    def item(self, out_np, i):
        return out_np[self.offs[i]:self.offs[i] + self.sizes[i]].astype(np.float64).reshape(self.shapes[i])


def _check_items(jt, orc, P, out_np, limit_of):
    worst = 0.0
    for i, (s, ab, d) in enumerate(zip(P.shapes, P.abs_, P.dirs)):
        got = P.item(out_np, i)
        x = P.xs_cast[i]
        ref = orc.forward(x, ab) if d == jt.FORWARD else orc.inverse(x, ab)
        e = relerr(got, ref)
        worst = max(worst, e)
        assert e <= limit_of(len(s)), (i, s, ab, d, e)
    return worst


# small multi-axis items run whole inside one block; (600, 900) and
# (70, 80, 90) are large enough to be split, so their later passes wait on
# device counters for the earlier ones
MIXED_SHAPES = [(100,), (64, 80), (300,), (5, 6, 7), (1,), (2048,), (33, 17), (1000,), (40, 130), (257,),
                (600, 900), (70, 80, 90)]
MIXED_AB = [((0.1, 0.2),), ((0.0, 0.1), (0.2, -0.2)), ((0.3, 0.3),), ((0.0, 0.1), (0.2, 0.2), (-0.3, 0.4)),
            ((0.1, 0.2),), ((0.2, 0.1),), ((0.1, 0.2), (0.3, -0.1)), ((0.25, -0.35),), ((-0.4, 0.1), (0.25, -0.35)),
            ((0.0, 0.0),), ((0.2, -0.1), (0.15, 0.05)), ((0.1, 0.1), (0.2, 0.2), (0.3, 0.3))]


@pytest.mark.parametrize("prec,tol", [(1, 1e-7), (0, 1e-12)])
def test_batch_mixed_items(jt, orc, prec, tol):
    dirs = [jt.FORWARD if i % 3 else jt.INVERSE for i in range(len(MIXED_SHAPES))]
    print("batch mixed prec=%d" % prec, flush=True)
    P = Prepared(jt, MIXED_SHAPES, MIXED_AB, dirs, tol, prec, seed=1)
    P.batch.run(P.inp, P.out)
    torch.cuda.synchronize()
    assert P.batch.errors() == 0
    floor = 1e-11 if prec == 0 else 2e-5
    w = _check_items(jt, orc, P, P.out.cpu().numpy(), lambda d: floor)
    print("worst item rel-l2 %.3e" % w)


@pytest.mark.parametrize("tin_name,tout_name", [("F32", "F64"), ("F64", "F32"), ("F32", "F32")])
def test_batch_dtypes(jt, orc, tin_name, tout_name):
    tin, tout = getattr(jt, tin_name), getattr(jt, tout_name)
    P = Prepared(jt, MIXED_SHAPES[:6], MIXED_AB[:6], [jt.FORWARD] * 6, 1e-7, 1, tin, tout, seed=2)
    P.batch.run(P.inp, P.out)
    torch.cuda.synchronize()
    assert P.batch.errors() == 0
    _check_items(jt, orc, P, P.out.cpu().numpy(), lambda d: 2e-5)


@pytest.mark.parametrize("opts", [{"max_split": 1}, {"min_units": 8}, {"grid": 3}])
def test_batch_tiling_options_give_the_same_results(jt, orc, opts):
    P = Prepared(jt, MIXED_SHAPES, MIXED_AB, [jt.FORWARD] * len(MIXED_SHAPES), 1e-7, 1, seed=3, **opts)
    P.batch.run(P.inp, P.out)
    torch.cuda.synchronize()
    assert P.batch.errors() == 0
    _check_items(jt, orc, P, P.out.cpu().numpy(), lambda d: 2e-5)


def test_batch_matches_the_single_transform_path(jt):
    P = Prepared(jt, MIXED_SHAPES, MIXED_AB, [jt.FORWARD] * len(MIXED_SHAPES), 1e-12, 0, seed=4)
    P.batch.run(P.inp, P.out)
    torch.cuda.synchronize()
    out = P.out.cpu().numpy()
    dev = _dev()
    for i, p in enumerate(P.plans):
        x = torch.from_numpy(P.xs[i]).to(dev)
        g = p.forward(x, prec=jt.PREC_FP64)
        torch.cuda.synchronize()
        assert relerr(P.item(out, i), g.cpu().numpy()) <= 1e-13


def test_batch_in_place(jt, orc):
    dev = _dev()
    shapes, abs_ = MIXED_SHAPES[:8], MIXED_AB[:8]
    P = Prepared(jt, shapes, abs_, [jt.INVERSE] * 8, 1e-7, 1, seed=5)
    buf = P.inp.clone()
    P.batch.run(buf, buf)
    torch.cuda.synchronize()
    _check_items(jt, orc, P, buf.cpu().numpy(), lambda d: 2e-5)
    assert dev.type == "cuda"


def test_batch_graph_replay_matches_eager(jt):
    P = Prepared(jt, MIXED_SHAPES, MIXED_AB, [jt.FORWARD if i % 2 else jt.INVERSE for i in range(12)], 1e-7, 1,
                 seed=6)
    P.batch.run(P.inp, P.out)
    torch.cuda.synchronize()
    eager = P.out.cpu().numpy().copy()
    P.batch.capture(P.inp, P.out)
    for rep in range(4):
        P.out.fill_(float("nan"))
        # unrelated eager work and a synchronisation between replays
        junk = torch.randn(1 << 20, device=P.out.device).sum()
        torch.cuda.synchronize()
        P.batch.replay()
        torch.cuda.synchronize()
        assert P.batch.errors() == 0
        assert np.array_equal(P.out.cpu().numpy(), eager), "replay %d differs" % rep
        del junk


def test_batch_ragged_1d_sample(jt, orc):
    """Items drawn like the 4096-item ragged 1D workload (n log-uniform in
    [64, 16384], (a, b) uniform in (-0.5, 0.5)), fp32 bulk, tol 1e-7, every
    item checked whole: against the long-double oracle up to n = 4096 and
    against its plain fp64 path above (the full 4096-item batch is checked in
    test_gpu_full_batch.py)."""
    items = workloads.batch_1d(48, seed=104)
    shapes = [(n,) for n, _, _ in items]
    abs_ = [(ab,) for _, ab, _ in items]
    xs = [x for _, _, x in items]
    dirs = [jt.FORWARD] * len(items)
    print("ragged 1d: sizes %s" % sorted(n for n, _, _ in items), flush=True)
    P = Prepared(jt, shapes, abs_, dirs, 1e-7, 1, xs=xs)
    P.batch.run(P.inp, P.out)
    torch.cuda.synchronize()
    assert P.batch.errors() == 0
    out = P.out.cpu().numpy()
    for i, (n, ab, x) in enumerate(items):
        got = P.item(out, i)
        ref = orc.forward(x, (ab,)) if n <= 4096 else orc.apply1d_fp64(x, ab)
        assert relerr(got, ref) <= 2e-5, (i, n)
    orc.clear_cache()


def test_batch_ragged_2d_sample(jt, orc):
    """Items drawn like the 4096-item ragged 2D workload (each n log-uniform
    in [32, 512]), forward and inverse mixed, fp32 bulk."""
    items = workloads.batch_2d(40, seed=1041)
    shapes = [n for n, _, _ in items]
    abs_ = [ab for _, ab, _ in items]
    xs = [x for _, _, x in items]
    dirs = [jt.FORWARD if i % 2 else jt.INVERSE for i in range(len(items))]
    P = Prepared(jt, shapes, abs_, dirs, 1e-7, 1, xs=xs)
    P.batch.run(P.inp, P.out)
    torch.cuda.synchronize()
    assert P.batch.errors() == 0
    _check_items(jt, orc, P, P.out.cpu().numpy(), lambda d: 2e-5)


def test_batch_round_trip_property(jt):
    """forward then inverse through two batches returns the input (the
    transform is orthogonal): a check that holds at any size."""
    items = workloads.batch_1d(24, seed=105)
    shapes = [(n,) for n, _, _ in items]
    abs_ = [(ab,) for _, ab, _ in items]
    xs = [x for _, _, x in items]
    F = Prepared(jt, shapes, abs_, [jt.FORWARD] * 24, 1e-7, 1, xs=xs)
    F.batch.run(F.inp, F.out)
    I = jt.Batch(F.plans, [jt.INVERSE] * 24, F.offs, F.offs, jt.F64, jt.F64, jt.PREC_FP32_BULK).bind(_dev())
    back = torch.empty_like(F.out)
    I.run(F.out, back)
    torch.cuda.synchronize()
    b = back.cpu().numpy()
    for i, x in enumerate(xs):
        assert relerr(F.item(b, i), x) <= 4e-5


LONG_SHAPES = [(16000,), (300,), (9000,), (16384,), (64, 80), (12000,)]
LONG_AB = [((0.2, -0.1),), ((0.1, 0.2),), ((-0.4, 0.3),), ((0.45, -0.45),), ((0.0, 0.1), (0.2, -0.2)), ((0.3, 0.3),)]


def _check_long(jt, orc, P, out_np):
    for i, (s, ab, d) in enumerate(zip(P.shapes, P.abs_, P.dirs)):
        x = P.xs_cast[i]
        if len(s) == 1 and s[0] > 4096:
            ref = orc.apply1d_fp64(x, ab[0], transpose=(d == jt.INVERSE))
        else:
            ref = orc.forward(x, ab) if d == jt.FORWARD else orc.inverse(x, ab)
        e = relerr(P.item(out_np, i), ref)
        assert e <= 2e-5, (i, s, d, e)


@pytest.mark.parametrize("tin_name,tout_name", [("F64", "F64"), ("F32", "F32")])
def test_batch_long_lines(jt, orc, tin_name, tout_name):
    """1D items of 8193 to 16384 points (one 16384-point line per block, two
    lanes per thread) beside short and multi-axis items: parity with the
    oracle in both directions and both dtypes, the same bits on every run, in
    place and on graph replays."""
    tin, tout = getattr(jt, tin_name), getattr(jt, tout_name)
    dirs = [jt.FORWARD if i % 2 else jt.INVERSE for i in range(len(LONG_SHAPES))]
    print("long lines %s -> %s" % (tin_name, tout_name), flush=True)
    P = Prepared(jt, LONG_SHAPES, LONG_AB, dirs, 1e-7, 1, tin, tout, seed=11)
    P.batch.run(P.inp, P.out)
    torch.cuda.synchronize()
    assert P.batch.errors() == 0
    first = P.out.cpu().numpy().copy()
    _check_long(jt, orc, P, first)
    for rep in range(3):
        P.out.fill_(float("nan"))
        P.batch.run(P.inp, P.out)
        torch.cuda.synchronize()
        assert np.array_equal(P.out.cpu().numpy(), first), "run %d differs" % rep
    if tin == tout:
        buf = P.inp.clone()
        P.batch.run(buf, buf)
        torch.cuda.synchronize()
        assert np.array_equal(buf.cpu().numpy(), first), "in place differs"
    P.batch.capture(P.inp, P.out)
    for rep in range(3):
        P.out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device=P.out.device).sum()
        torch.cuda.synchronize()
        P.batch.replay()
        torch.cuda.synchronize()
        assert P.batch.errors() == 0
        assert np.array_equal(P.out.cpu().numpy(), first), "replay %d differs" % rep
        del junk
    orc.clear_cache()
