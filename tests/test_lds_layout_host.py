"""Host checks of the inverse direct block's LDS layout and the nu0 cap.

The axis pass (one-pass and persistent kernels) reuses a line buffer of
L + L/16 complex values for the inverse direct block (alpha_k for k < nu0,
eq. (51)): the per-degree sums red[0, nu0) (rounded up to 16 bytes), then
line_sum's per-wave partials when a line spans several waves, then the staged
line of L values when n is a multiple of 4 and it fits.  This walks every
kernel instantiation (line length, lanes per thread, precision) and every
accepted nu0 and checks that the regions are disjoint and inside the buffer,
with the same formulas the kernel uses.  No GPU is involved.
"""
import pytest

import paper_1901_07275_amd as jt

MAX_NU0 = 64
BATCH_THREADS = 512


def geo(log2l, vl=1):
    L = 1 << log2l
    P = L // 16
    tpl = P // vl
    block = 64 if tpl < 64 else tpl
    return L, P, tpl, block


def instantiations():
    out = []
    for tsize in (4, 8):
        for log2l in range(6, 15):
            if tsize == 8 and log2l > 13:
                continue  # fp64 lines stop at 8192 points
            out.append((tsize, log2l, 1))  # one-pass kernel
            P = (1 << log2l) // 16
            vl = P // BATCH_THREADS if P > BATCH_THREADS else 1
            out.append((tsize, log2l, vl))  # persistent kernel
    return sorted(set(out))


@pytest.mark.parametrize("tsize,log2l,vl", instantiations())
def test_inverse_direct_block_regions_are_disjoint(tsize, log2l, vl):
    L, P, tpl, _ = geo(log2l, vl)
    _, _, _, block1 = geo(log2l)  # the chunk width follows the one-lane geometry
    kc = 8 if block1 <= 256 else 2
    buf_bytes = (L + L // 16) * 2 * tsize
    lsum_n = (tpl // 64) * kc if tpl > 64 else 0
    for nu0 in range(1, MAX_NU0 + 1):
        if nu0 > L:
            continue
        red_n = (nu0 + 1) & ~1
        red = (0, 8 * nu0)
        lsum = (8 * red_n, 8 * (red_n + lsum_n))
        gs_off = 8 * (red_n + lsum_n)
        assert gs_off % 16 == 0
        assert red[1] <= lsum[0]
        assert lsum[1] <= buf_bytes, (nu0, lsum, buf_bytes)
        staged = gs_off + L * tsize <= buf_bytes
        if staged:
            assert gs_off >= lsum[1] and gs_off + L * tsize <= buf_bytes
        # the staged line always fits except on the shortest fp32 lines with a wide block
        if not staged:
            assert tsize == 4 and L == 64 and nu0 > 36, (tsize, L, nu0)
        # the S > 1 partial sums (L doubles) fit in one line buffer
        assert 8 * L <= buf_bytes


def test_plan_rejects_direct_blocks_wider_than_64():
    with pytest.raises(jt.JTError) as e:
        jt.Plan((256,), ((0.1, 0.2),), 1e-8, nu0=65)
    assert e.value.status == jt.JT_EINVAL
    assert "nu0" in str(e.value)
    p = jt.Plan((256,), ((0.1, 0.2),), 1e-8, nu0=64)
    assert p.info(0)["nu0"] == 64
