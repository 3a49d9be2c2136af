"""The batch entry point that allocates nothing (jt_batch_run_static): its
counters live in the library's own device array instead of the batch's bound
buffer.  Through the C ABI, two calls in a row (the second on a smaller
batch, so the array holds the first call's counters when it starts) must give
exactly what jt_batch_run gives on the same batches; the error word reaches
jt_batch_errors; a batch with more axis passes than the array holds is
rejected before anything runs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(100,), (64, 80), (300,), (5, 6, 7), (2048,), (600, 900), (70, 80, 90), (1000,), (40, 130)]
AB = [((0.1, 0.2),), ((0.0, 0.1), (0.2, -0.2)), ((0.3, 0.3),), ((0.0, 0.1), (0.2, 0.2), (-0.3, 0.4)),
      ((0.2, 0.1),), ((0.2, -0.1), (0.15, 0.05)), ((0.1, 0.1), (0.2, 0.2), (0.3, 0.3)), ((0.25, -0.35),),
      ((-0.4, 0.1), (0.25, -0.35))]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def jt():
    import paper_1901_07275_amd as m

    return m


def _batch(jt, shapes, abs_, prec, seed):
    dev = _dev()
    plans = jt.plan_many(shapes, abs_, 1e-7 if prec == jt.PREC_FP32_BULK else 1e-12)
    arena = jt.PlanArena(plans, dev)
    sizes = [int(np.prod(s)) for s in shapes]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)
    dirs = [jt.FORWARD if i % 3 else jt.INVERSE for i in range(len(shapes))]
    B = jt.Batch(plans, dirs, offs, offs, jt.F64, jt.F64, prec).bind(dev)
    rng = np.random.default_rng(seed)
    inp = torch.from_numpy(np.concatenate([rng.standard_normal(s).ravel() for s in shapes])).to(dev)
    return B, arena, inp


@pytest.mark.parametrize("prec", [1, 0])
def test_static_counters_match_the_bound_counters(jt, prec):
    big = _batch(jt, SHAPES, AB, prec, 1)
    small = _batch(jt, SHAPES[:4], AB[:4], prec, 2)
    for B, arena, inp in (big, small):  # two calls in a row, the second smaller
        ref = torch.full_like(inp, float("nan"))
        B.run(inp, ref)
        torch.cuda.synchronize()
        assert B.errors() == 0
        out = torch.full_like(inp, float("nan"))
        B.run_static(inp, out)
        torch.cuda.synchronize()
        assert B.errors() == 0
        assert torch.equal(out, ref)
    # and again on the large batch after the small one left its counters behind
    B, arena, inp = big
    out = torch.full_like(inp, float("nan"))
    B.run_static(inp, out)
    B.run_static(inp, out)
    torch.cuda.synchronize()
    ref = torch.full_like(inp, float("nan"))
    B.run(inp, ref)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert B.errors() == 0


def test_static_counters_reject_too_many_passes(jt):
    """65535 one-axis items need 65537 counter words, one more than the array
    holds: refused before anything is launched (the batch is not even bound)."""
    count = 65535
    plans = jt.plan_many([(1,)] * count, [((0.0, 0.0),)] * count, 1e-7)
    offs = np.arange(count)
    B = jt.Batch(plans, [jt.FORWARD] * count, offs, offs, jt.F64, jt.F64, jt.PREC_FP32_BULK)
    x = torch.zeros(count, dtype=torch.float64, device=_dev())
    with pytest.raises(jt.JTError) as e:
        B.run_static(x, x)
    assert e.value.status == jt.JT_EINVAL
    assert "65534" in str(e.value)
