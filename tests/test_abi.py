"""The C ABI (no GPU): every symbol include/jt.h declares is exported, and
argument errors come back as status codes with a message."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1901_07275_amd as jt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "jt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(jt_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(jt.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 27
    for name in names:
        assert hasattr(lib, name), name
    assert set(jt.SYMBOLS) | {"jt_last_error", "jt_version", "jt_clock"} >= set(names)


def test_version():
    assert jt.version() == 124


@pytest.mark.parametrize("n,ab,tol", [
    ([], [], 1e-8),
    ([0], [(0.1, 0.1)], 1e-8),
    ([100], [(-1.0, 0.1)], 1e-8),
    ([100], [(0.1, 1.0)], 1e-8),
    ([100], [(0.1, 0.1)], 1.0),
    ([100], [(0.1, 0.1)], 1e-16),
    ([20000], [(0.1, 0.1)], 1e-8),
    ([4, 4, 4, 4], [(0.1, 0.1)] * 4, 1e-8),
])
def test_plan_rejects_bad_arguments(n, ab, tol):
    with pytest.raises(jt.JTError) as e:
        jt.Plan(n, ab, tol)
    assert e.value.status == jt.JT_EINVAL
    assert str(e.value)


def test_unbound_plan_refuses_transforms():
    P = jt.Plan([64], [(0.1, 0.2)], 1e-8)
    st = jt._lib.jt_forward(P._h, jt._vp(16), 0, jt._vp(32), 0, 0, jt._vp(0))
    assert st == jt.JT_ESTATE
    assert b"bind" in jt._lib.jt_last_error()


def test_bind_checks_size_and_alignment():
    P = jt.Plan([64], [(0.1, 0.2)], 1e-8)
    nb = P.device_bytes()
    assert jt._lib.jt_plan_bind(P._h, jt._vp(256), nb - 1, jt._vp(0)) == jt.JT_ENOMEM
    assert jt._lib.jt_plan_bind(P._h, jt._vp(257), nb, jt._vp(0)) == jt.JT_EINVAL


def test_info_and_axis_checks():
    P = jt.Plan([100, 64], [(0.1, 0.2), (0.3, 0.1)], 1e-8)
    d = ctypes.c_int()
    assert jt._lib.jt_plan_dims(P._h, ctypes.byref(d)) == jt.JT_OK and d.value == 2
    with pytest.raises(jt.JTError):
        P.info(2)
    with pytest.raises(jt.JTError):
        P.entries(0, [0], [3])  # degree below nu0
    ws = ctypes.c_size_t(123)
    assert jt._lib.jt_workspace_bytes(P._h, 0, ctypes.byref(ws)) == jt.JT_OK and ws.value == 0
    img = P.pack()
    assert img.nbytes == P.device_bytes() and img.nbytes % 256 == 0
