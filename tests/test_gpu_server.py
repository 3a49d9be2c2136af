"""GPU tests of the serving form (continuous batching over a device arena).

Each result must match the oracle (fp32 bulk at tol 1e-7: 2e-5 rel-l2), and
must be bit-for-bit the same whether the request ran alone or in a mix: a
unit's arithmetic does not depend on the other requests of its launch.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def jt():
    import paper_1901_07275_amd as m

    return m


def relerr(x, ref):
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


REQS = [((100,), ((0.1, 0.2),), 0), ((40, 70), ((0.0, 0.1), (0.2, -0.2)), 1), ((300,), ((0.3, 0.3),), 0),
        ((5, 6, 7), ((0.0, 0.1), (0.2, 0.2), (-0.3, 0.4)), 0), ((33, 17), ((0.1, 0.2), (0.3, -0.1)), 0),
        ((100,), ((0.1, 0.2),), 1), ((2000,), ((0.25, -0.35),), 0), ((64, 64, 64), ((0.3, 0.3),) * 3, 1),
        ((1024, 300), ((0.25, -0.35), (-0.4, 0.1)), 0)]


def _oracle(orc, x, ab, direction):
    x = x.astype(np.float64)
    return orc.forward(x, ab) if direction == 0 else orc.inverse(x, ab)


def _inputs(seed=5):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s).astype(np.float32) for s, _, _ in REQS]


def test_server_alone_matches_oracle_and_mix_is_bitwise_equal(jt, orc):
    _need_gpu()
    xs = _inputs()
    S = jt.Server(64 << 20)
    alone = []
    for (s, ab, d), x in zip(REQS, xs):
        out = np.full(s, np.nan, np.float32)
        info = S.wait(S.submit(x, out, ab, d))
        assert info["state"] == 3
        e = relerr(out, _oracle(orc, x, ab, d))
        print("alone", s, "rel-l2 %.2e" % e, "cold", info["cold"], flush=True)
        assert e <= 2e-5
        alone.append(out.copy())
    st = S.stats()
    assert st["completed"] == len(REQS) and st["failed"] == 0
    # the same requests three times over, interleaved, submitted at once
    outs, tickets = [], []
    for rep in range(3):
        for i, ((s, ab, d), x) in enumerate(zip(REQS, xs)):
            out = np.full(s, np.nan, np.float32)
            outs.append((i, out))
            tickets.append(S.submit(x, out, ab, d))
    infos = [S.wait(t) for t in tickets]
    assert all(inf["state"] == 3 for inf in infos)
    for i, out in outs:
        assert np.array_equal(out, alone[i]), "request %d differs between alone and mix" % i
    st = S.stats()
    assert st["launches"] < len(REQS) + 3 * len(REQS), "the mix should share launches"
    assert st["plan_hits"] > 0
    S.close()


def test_server_admission_in_a_small_arena(jt, orc):
    """An arena that holds only a few requests at a time: requests wait for
    memory, plans are evicted and rebuilt, and every result is still right."""
    _need_gpu()
    xs = _inputs(7)
    S = jt.Server(6 << 20, max_batch=4)
    outs, tickets = [], []
    for rep in range(2):
        for i, ((s, ab, d), x) in enumerate(zip(REQS, xs)):
            out = np.full(s, np.nan, np.float32)
            outs.append((i, out))
            tickets.append(S.submit(x, out, ab, d))
    for t in tickets:
        S.wait(t)
    st = S.stats()
    print("small arena stats", st, flush=True)
    assert st["arena_peak"] <= st["arena_bytes"]
    assert st["failed"] == 0
    for i, out in outs:
        s, ab, d = REQS[i]
        assert relerr(out, _oracle(orc, xs[i], ab, d)) <= 2e-5
    S.close()


def test_server_rejects_a_request_larger_than_the_arena(jt):
    _need_gpu()
    S = jt.Server(1 << 20)
    x = np.zeros((512, 512), np.float32)
    out = np.zeros_like(x)
    with pytest.raises(jt.JTError) as e:
        S.submit(x, out, ((0.1, 0.1), (0.1, 0.1)))
    assert e.value.status == jt.JT_ENOMEM
    S.close()


def test_server_plan_cache_hits_are_warm(jt):
    _need_gpu()
    S = jt.Server(32 << 20)
    x = np.random.default_rng(1).standard_normal(777).astype(np.float32)
    o1, o2 = np.zeros_like(x), np.zeros_like(x)
    i1 = S.wait(S.submit(x, o1, ((0.2, -0.1),)))
    i2 = S.wait(S.submit(x, o2, ((0.2, -0.1),)))
    assert i1["cold"] == 1 and i2["cold"] == 0
    assert i1["plan_seconds"] > 0 and i2["plan_seconds"] == 0
    assert np.array_equal(o1, o2)
    assert i2["t_submit"] <= i2["t_admit"] <= i2["t_launch"] <= i2["t_done"]
    S.close()


def test_server_fp64(jt, orc):
    _need_gpu()
    S = jt.Server(64 << 20, tol=1e-12, prec=jt.PREC_FP64, dtype=jt.F64)
    rng = np.random.default_rng(3)
    for s, ab, d in REQS[:6]:
        x = rng.standard_normal(s)
        out = np.zeros(s)
        S.wait(S.submit(x, out, ab, d))
        assert relerr(out, _oracle(orc, x, ab, d)) <= 1e-11
    S.close()


def test_server_mixed_stream_sample(jt, orc):
    """A short stretch of the mixed serving stream (d = 1, 2, 3, sizes and
    (a, b) as in the serving workload), submitted with Poisson gaps."""
    _need_gpu()
    import time

    reqs = workloads.serving_stream(40, seed=105)
    rng = np.random.default_rng(9)
    xs = [rng.standard_normal(s).astype(np.float32) for _, s, _, _ in reqs]
    S = jt.Server(2 << 30)
    arrivals = workloads.poisson_arrivals(len(reqs), 200.0)
    t0 = time.monotonic()
    outs, tickets = [], []
    for (d, s, ab, direction), x, ta in zip(reqs, xs, arrivals):
        delay = t0 + ta - time.monotonic()
        if delay > 0:
            time.sleep(delay)
        out = np.full(s, np.nan, np.float32)
        outs.append(out)
        tickets.append(S.submit(x, out, ab, direction))
    infos = [S.wait(t) for t in tickets]
    assert all(inf["state"] == 3 for inf in infos)
    big = 0
    for k, ((d, s, ab, direction), x, out) in enumerate(zip(reqs, xs, outs)):
        if int(np.prod(s)) <= 1 << 20:
            assert relerr(out, _oracle(orc, x, ab, direction)) <= 2e-5
        else:
            # 256 outputs, each computed on its own by the oracle; their
            # rel-l2 against the sample's norm (entries are O(|x| / sqrt(N)))
            big += 1
            idx = np.random.default_rng(k).integers(0, np.array(s), size=(256, len(s)))
            f = orc.forward_entries if direction == 0 else orc.inverse_entries
            ref = f(x.astype(np.float64), ab, idx)
            assert relerr(out[tuple(idx.T)].astype(np.float64), ref) <= 2e-5, (k, s)
            assert abs(np.linalg.norm(out) / np.linalg.norm(x) - 1) <= 1e-4
    print("requests above 2^20 coefficients checked on samples: %d" % big)
    st = S.stats()
    print("stream stats", st, flush=True)
    S.close()


def test_server_dense_crossover_per_regime(jt, orc):
    """dense_below applies to multi-axis requests and dense_below_1d to 1D
    ones: an axis of the same n is planned both ways (two cache entries)
    and both results match the oracle."""
    _need_gpu()
    S = jt.Server(64 << 20, dense_below=300, dense_below_1d=100)
    rng = np.random.default_rng(11)
    cases = [((200,), ((0.1, 0.2),)), ((200, 40), ((0.1, 0.2), (0.3, -0.1)))]
    for s, ab in cases:
        x = rng.standard_normal(s).astype(np.float32)
        out = np.full(s, np.nan, np.float32)
        S.wait(S.submit(x, out, ab))
        assert relerr(out, _oracle(orc, x, ab, 0)) <= 2e-5
    st = S.stats()
    # n = 200 twice (FFT for the 1D request, dense for the 2D one) and n = 40
    assert st["plans_cached"] == 3 and st["plan_misses"] == 3
    S.close()
