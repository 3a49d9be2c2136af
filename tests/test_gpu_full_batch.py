"""The two 4096-item ragged batches at full size, in the launch configuration
the benchmark times (tuned FFT-versus-dense crossover per item, tuned split
cap, fp32 bulk with fp32 input and output, one persistent launch replayed
from a captured HIP graph), every item checked whole against the oracle.

  * 1D: n log-uniform in [64, 16384], (a, b) uniform in (-1/2, 1/2), tol 1e-7.
    The oracle side is its plain fp64 path (nodes by safeguarded Newton,
    the sums by the recurrence), pinned to the long-double construction;
    its own error (below 1e-9) is far under the bar.
  * 2D: n0, n1 log-uniform in [32, 512], forward and inverse mixed.

Bar: rel-l2 <= 2e-5 per item (fp32 bulk at tol 1e-7; Section 3.1 eqs.
(50)-(51) per item, Section 3.2 for the 2D items).  A replay of the captured
graph must equal the eager launch bit for bit.

The host planning of 4096 items and the oracle's 4096 transforms take
minutes, so both are cut into chunks of 512 items, one test each, run in file
order and sharing a module-level cache (a chunk test run on its own builds
whatever it needs).
"""
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COUNT, CHUNK = 4096, 512
CHUNKS = list(range(COUNT // CHUNK))


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


class FullBatch:
    def __init__(self, kind):
        if kind == "1d":
            items = workloads.batch_1d(COUNT, seed=104)
            self.shapes = [(n,) for n, _, _ in items]
            self.abs_ = [(ab,) for _, ab, _ in items]
            self.dirs = [0] * COUNT
        else:
            items = workloads.batch_2d(COUNT, seed=1041)
            self.shapes = [n for n, _, _ in items]
            self.abs_ = [ab for _, ab, _ in items]
            self.dirs = [1 - i % 2 for i in range(COUNT)]  # inverse, forward, ...
        self.xs = [x for _, _, x in items]
        self.plans = {}
        self.out = None

    def plan_chunk(self, jt, c):
        if c in self.plans:
            return
        from paper_1901_07275_amd import autotune

        tuning = autotune.load()
        sl = slice(c * CHUNK, (c + 1) * CHUNK)
        db = [autotune.dense_below(1 if len(s) == 1 else min(s), jt.PREC_FP32_BULK, tuning)
              for s in self.shapes[sl]]
        t0 = time.perf_counter()
        self.plans[c] = jt.plan_many(self.shapes[sl], self.abs_[sl], 1e-7, dense_below=db)
        print("chunk %d planned in %.1f s" % (c, time.perf_counter() - t0))

    def output(self, jt):
        if self.out is not None:
            return self.out
        from paper_1901_07275_amd import autotune

        for c in CHUNKS:
            self.plan_chunk(jt, c)
        dev = _dev()
        plans = [p for c in CHUNKS for p in self.plans[c]]
        arena = jt.PlanArena(plans, dev)
        self.sizes = [int(np.prod(s)) for s in self.shapes]
        self.offs = np.concatenate([[0], np.cumsum(self.sizes)[:-1]]).astype(int)
        B = jt.Batch(plans, self.dirs, self.offs, self.offs, jt.F32, jt.F32, jt.PREC_FP32_BULK,
                     max_split=int(autotune.load().get("max_split", 0))).bind(dev)
        inp = torch.from_numpy(np.concatenate([x.ravel() for x in self.xs])).to(dev, torch.float32)
        out = torch.full_like(inp, float("nan"))
        print("batch: %d items, %d coefficients, %d units" % (COUNT, sum(self.sizes), B.info()["units"]))
        B.run(inp, out)
        torch.cuda.synchronize()
        assert B.errors() == 0
        eager = out.cpu().numpy().copy()
        B.capture(inp, out)
        out.fill_(float("nan"))
        B.replay()
        torch.cuda.synchronize()
        assert B.errors() == 0
        assert np.array_equal(out.cpu().numpy(), eager)
        del B, arena
        self.out = eager
        return eager

    def item(self, i):
        return self.out[self.offs[i]:self.offs[i] + self.sizes[i]].astype(np.float64).reshape(self.shapes[i])


_batches = {}


def _batch(kind):
    if kind not in _batches:
        _batches[kind] = FullBatch(kind)
    return _batches[kind]


@pytest.mark.parametrize("c", CHUNKS)
def test_full_1d_plan(jt, c):
    _batch("1d").plan_chunk(jt, c)


def test_full_1d_run(jt):
    _batch("1d").output(jt)


@pytest.mark.parametrize("c", CHUNKS)
def test_full_1d_items(jt, orc, c):
    fb = _batch("1d")
    fb.output(jt)
    worst = 0.0
    for i in range(c * CHUNK, (c + 1) * CHUNK):
        x32 = fb.xs[i].astype(np.float32).astype(np.float64)
        ref = orc.apply1d_fp64(x32, fb.abs_[i][0])
        e = relerr(fb.item(i), ref)
        worst = max(worst, e)
        assert e <= 2e-5, (i, fb.shapes[i], fb.abs_[i], e)
    print("1D items %d..%d: worst rel-l2 %.3e" % (c * CHUNK, (c + 1) * CHUNK - 1, worst))


@pytest.mark.parametrize("c", CHUNKS)
def test_full_2d_items(jt, orc, c):
    fb = _batch("2d")
    fb.output(jt)
    worst = 0.0
    for i in range(c * CHUNK, (c + 1) * CHUNK):
        x32 = fb.xs[i].astype(np.float32).astype(np.float64)
        ref = orc.forward(x32, fb.abs_[i]) if fb.dirs[i] == 0 else orc.inverse(x32, fb.abs_[i])
        e = relerr(fb.item(i), ref)
        worst = max(worst, e)
        assert e <= 2e-5, (i, fb.shapes[i], fb.abs_[i], fb.dirs[i], e)
    orc.clear_cache()
    print("2D items %d..%d: worst rel-l2 %.3e" % (c * CHUNK, (c + 1) * CHUNK - 1, worst))


def test_full_batches_release_memory():
    _batches.clear()
