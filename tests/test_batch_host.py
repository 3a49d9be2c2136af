"""Host logic of the batched form (no GPU): many plans at once, and the
work-unit queue that the persistent kernel consumes."""
import numpy as np
import pytest

import paper_1901_07275_amd as jt
import workloads


def _items():
    shapes = [(100,), (64, 80), (300,), (5, 6, 7), (1,), (2048,), (33, 17), (800, 700), (70, 80, 90)]
    abs_ = [((0.1, 0.2),), ((0.0, 0.1), (0.2, -0.2)), ((0.3, 0.3),), ((0.0, 0.1), (0.2, 0.2), (-0.3, 0.4)),
            ((0.1, 0.2),), ((0.2, 0.1),), ((0.1, 0.2), (0.3, -0.1)), ((0.1, 0.1), (0.2, 0.2)),
            ((0.1, 0.1), (0.2, 0.2), (0.3, 0.3))]
    return shapes, abs_


def test_plan_many_matches_single_plans():
    shapes, abs_ = _items()
    many = jt.plan_many(shapes, abs_, 1e-7)
    for s, ab, p in zip(shapes, abs_, many):
        one = jt.Plan(s, ab, 1e-7)
        assert p.n == tuple(s)
        assert np.array_equal(p.pack(), one.pack())


def test_plan_many_reports_the_failing_item():
    with pytest.raises(jt.JTError) as e:
        jt.plan_many([(10,), (0,)], [((0.1, 0.1),), ((0.1, 0.1),)], 1e-7)
    assert e.value.status == jt.JT_EINVAL
    assert "item 1" in str(e.value)


def _offsets(shapes):
    sizes = [int(np.prod(s)) for s in shapes]
    return np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)


@pytest.mark.parametrize("prec", [jt.PREC_FP32_BULK, jt.PREC_FP64])
@pytest.mark.parametrize("opts", [{}, {"max_split": 1}, {"min_units": 8}, {"max_split": 4, "min_units": 2}])
def test_unit_table_covers_every_line_once(prec, opts):
    shapes, abs_ = _items()
    plans = jt.plan_many(shapes, abs_, 1e-7)
    offs = _offsets(shapes)
    dirs = [jt.FORWARD if i % 2 else jt.INVERSE for i in range(len(shapes))]
    B = jt.Batch(plans, dirs, offs, offs, jt.F64, jt.F64, prec, **opts)
    units, passes = B.tables()
    info = B.info()
    assert info["units"] == len(units) and info["passes"] == len(passes) == sum(len(s) for s in shapes)
    assert info["threads"] == 512
    assert info["lds_bytes"] == 139264 + 16
    covered = {p: np.zeros(passes[p, 2], dtype=int) for p in range(len(passes))}
    for pid, line0, nl, split, wp, wc, npass in units:
        if npass > 0:  # a whole small item: every line of its passes
            assert wp == -1 and npass == len(shapes[passes[pid, 0]])
            for p in range(pid, pid + npass):
                assert passes[p, 0] == passes[pid, 0]
                covered[p][:] += 1
            continue
        assert nl >= 1 and split >= 1 and (split & (split - 1)) == 0
        if opts.get("max_split"):
            assert split <= opts["max_split"]
        covered[pid][line0:line0 + nl] += 1
    for p, c in covered.items():
        assert np.all(c == 1), "pass %d lines not covered exactly once" % p
    # unit counts per pass, and each item's passes run along axes d-1 .. 0
    for p in range(len(passes)):
        assert passes[p, 3] == np.sum(units[:, 0] == p)
    pos = 0
    for i, s in enumerate(shapes):
        assert list(passes[pos:pos + len(s), 0]) == [i] * len(s)
        assert list(passes[pos:pos + len(s), 1]) == list(range(len(s) - 1, -1, -1))
        pos += len(s)


def test_waits_point_to_the_previous_pass_and_queue_order_is_safe():
    shapes, abs_ = _items()
    plans = jt.plan_many(shapes, abs_, 1e-7)
    offs = _offsets(shapes)
    # a grid of one block: every small multi-axis item is within the share
    B = jt.Batch(plans, [jt.FORWARD] * len(shapes), offs, offs, grid=1)
    units, passes = B.tables()
    first_pos = {}
    for q, (pid, *_rest) in enumerate(units):
        first_pos.setdefault(pid, q)
    last_pos = {pid: q for q, (pid, *_rest) in enumerate(units)}
    fused_items = {passes[pid, 0] for pid, *_r, npass in units if npass > 0}
    # small multi-axis items run whole; the large ones are split and wait
    assert fused_items == {i for i, s in enumerate(shapes) if len(s) > 1 and len(s) * np.prod(s) <= 1 << 19}
    for q, (pid, line0, nl, split, wp, wc, npass) in enumerate(units):
        item, axis = passes[pid, 0], passes[pid, 1]
        d = len(shapes[item])
        if npass > 0 or axis == d - 1:
            assert wp == -1 and wc == 0
        else:
            assert passes[wp, 0] == item and passes[wp, 1] == axis + 1
            assert wc == passes[wp, 3]
            # every unit waited for sits earlier in the queue (no deadlock)
            assert last_pos[wp] < q


def test_fusion_keeps_the_batch_critical_path():
    """A small multi-axis item runs whole in one block only while that does
    not lengthen the batch: its fused work stays within the work per block or
    the longest critical path of a split item.  Many tiny items fuse, a few
    mid-size ones (many units per pass) are split across blocks, and items
    whose passes are one unit each fuse however few they are."""
    def fused(shapes, **kw):
        distinct = sorted(set(shapes))
        one = dict(zip(distinct, jt.plan_many(distinct, [tuple((0.1, 0.1) for _ in s) for s in distinct], 1e-7)))
        plans = [one[s] for s in shapes]
        offs = _offsets(shapes)
        units, passes = jt.Batch(plans, [jt.FORWARD] * len(shapes), offs, offs, **kw).tables()
        return {passes[pid, 0] for pid, *_r, npass in units if npass > 0}

    assert fused([(8, 8)] * 600) == set(range(600))
    assert fused([(300, 300)] * 4) == set()
    assert fused([(300, 300)] * 4, grid=1) == set(range(4))
    # one mid-size item among many tiny ones is split, the tiny ones fuse
    mixed = [(8, 8)] * 300 + [(300, 300)]
    assert fused(mixed) == set(range(300))
    # one unit per pass (lines of 40 points: 128 lines per unit): nothing to split
    assert fused([(30, 40)] * 4) == set(range(4))


def test_batch_rejects_bad_arguments():
    p64 = jt.plan_many([(9000,)], [((0.1, 0.1),)], 1e-7)
    with pytest.raises(jt.JTError) as e:
        jt.Batch(p64, [jt.FORWARD], [0], [0], prec=jt.PREC_FP64)
    assert e.value.status == jt.JT_EUNSUPPORTED
    plans = jt.plan_many([(10,)], [((0.1, 0.1),)], 1e-7)
    with pytest.raises(jt.JTError):
        jt.Batch(plans, [7], [0], [0])
    with pytest.raises(jt.JTError):
        jt.Batch(plans, [jt.FORWARD], [0], [0], max_split=-1)
    # misaligned byte offset is impossible through element offsets; check the raw ABI
    import ctypes

    h = ctypes.c_void_p()
    hs = (ctypes.c_void_p * 1)(plans[0]._h.value)
    st = jt._lib.jt_batch_create(1, ctypes.cast(hs, ctypes.c_void_p), (ctypes.c_int * 1)(0),
                                 (ctypes.c_uint64 * 1)(4), (ctypes.c_uint64 * 1)(0), jt.F64, jt.F64, 1, None,
                                 ctypes.byref(h))
    assert st == jt.JT_EINVAL
    st = jt._lib.jt_batch_create(0, None, None, None, None, jt.F64, jt.F64, 1, None, ctypes.byref(h))
    assert st == jt.JT_EINVAL


def test_unbound_batch_cannot_run():
    plans = jt.plan_many([(10,)], [((0.1, 0.1),)], 1e-7)
    B = jt.Batch(plans, [jt.FORWARD], [0], [0])
    import ctypes

    st = jt._lib.jt_batch_run(B._h, ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert st == jt.JT_ESTATE
    st = jt._lib.jt_batch_replay(B._h, None)
    assert st == jt.JT_ESTATE


def test_single_line_items_get_the_rank_split():
    """A 1D item is one line: its rank terms are spread over the block's groups."""
    plans = jt.plan_many([(1000,), (16000,)], [((0.1, 0.2),), ((0.2, -0.1),)], 1e-7)
    B = jt.Batch(plans, [jt.FORWARD] * 2, [0, 1000], [0, 1000])
    units, passes = B.tables()
    by_pass = {int(u[0]): u for u in units}
    r0 = plans[0].info(0)["rank"]
    # L = 1024: 8 single-wave groups in a 512-thread block
    assert by_pass[0][3] == min(8, 1 << int(np.ceil(np.log2(r0))))
    # L = 16384: one group of 512 threads with two lanes each, no split possible
    assert by_pass[1][3] == 1


def test_batched_workload_recipe_is_seeded():
    a = workloads.batch_1d(8)
    b = workloads.batch_1d(8)
    assert [x[0] for x in a] == [x[0] for x in b]
    assert all(64 <= x[0] <= 16384 for x in a)
    c = workloads.batch_2d(8)
    assert all(32 <= m <= 512 for x in c for m in x[0])


def test_dense_units_hold_as_many_lines_as_lds_allows():
    """A dense (matrix-core) unit stages 64, 32 or 16 lines: the most whose
    rows fit the block's 139264 bytes of LDS, and no more than the pass has."""
    def rows(n, elem, lines):
        r = 64
        while r > 16 and (r * (n | 1) * elem > 139264 or r // 2 >= lines):
            r //= 2
        return r

    shapes = [(1000, 300), (7, 500)]
    abs_ = [((0.1, 0.2), (0.3, -0.1)), ((0.2, 0.2), (0.1, 0.0))]
    for prec, elem in ((jt.PREC_FP32_BULK, 4), (jt.PREC_FP64, 8)):
        plans = jt.plan_many(shapes, abs_, 1e-7, dense_below=[1025, 1025])
        offs = _offsets(shapes)
        units, passes = jt.Batch(plans, [jt.FORWARD] * 2, offs, offs, jt.F64, jt.F64, prec, grid=256).tables()
        seen = 0
        for pid in range(len(passes)):
            item, axis = passes[pid, 0], passes[pid, 1]
            s = shapes[item]
            n, lines = s[axis], int(np.prod(s)) // s[axis]
            mine = units[units[:, 0] == pid]
            if len(mine) == 0 or mine[0, 6] > 0:
                continue  # fused into one unit
            want = rows(n, elem, lines)
            assert np.all(mine[:-1, 2] == want) and 1 <= mine[-1, 2] <= want, (prec, s, axis)
            assert mine[:, 2].sum() == lines
            seen += 1
        assert seen >= 2
