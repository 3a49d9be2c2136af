"""Python binding of the MI355X fast multi-dimensional Jacobi transform.

Thin ctypes marshalling over the C ABI in include/jt.h (libjt.so, built
in-tree by ``paper_1901_07275_amd.build``).  Every step of the transform runs
in the library's HIP kernels; torch is used only to hold device memory and
to name the stream.  There is no CPU fallback: if libjt.so is missing the
import fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libjt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libjt.so not found at %s; build it with `python paper_1901_07275_amd/build.py`" % LIB_PATH)

# torch first: libjt.so then binds to the HIP runtime torch already loaded
# (same soname), so tensors, streams and kernels share one runtime.  Loading
# libjt.so first would bring in a second HIP/HSA runtime beside torch's.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)


def _hip_runtimes() -> set:
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return {line.split()[-1] for line in f if "libamdhip64" in line}
    except OSError:
        return set()


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are loaded (%s); import torch before anything that loads "
                      "/opt/rocm's libamdhip64" % ", ".join(sorted(_hip_runtimes())))

JT_OK, JT_EINVAL, JT_ENOMEM, JT_EDEVICE, JT_ENOTCONV, JT_EUNSUPPORTED, JT_ESTATE = range(7)
F64, F32 = 0, 1
PREC_FP64, PREC_FP32_BULK = 0, 1
FORWARD, INVERSE = 0, 1
_STATUS = {0: "JT_OK", 1: "JT_EINVAL", 2: "JT_ENOMEM", 3: "JT_EDEVICE", 4: "JT_ENOTCONV",
           5: "JT_EUNSUPPORTED", 6: "JT_ESTATE"}


class PlanOptions(ctypes.Structure):
    _fields_ = [("nu0", ctypes.c_int), ("dense_below", ctypes.c_int), ("oversample", ctypes.c_int),
                ("iterations", ctypes.c_int), ("seed", ctypes.c_uint64), ("kind", ctypes.c_int),
                ("planner", ctypes.c_int)]


class AxisInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("L", ctypes.c_int), ("nu0", ctypes.c_int), ("rank", ctypes.c_int),
                ("max_per_bin", ctypes.c_int), ("rsvd_rounds", ctypes.c_int),
                ("rel_err", ctypes.c_double), ("fro", ctypes.c_double), ("planner", ctypes.c_int)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("max_split", ctypes.c_int), ("min_units", ctypes.c_int), ("grid", ctypes.c_int)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("units", ctypes.c_int), ("passes", ctypes.c_int), ("grid", ctypes.c_int),
                ("threads", ctypes.c_int), ("lds_bytes", ctypes.c_size_t), ("cost", ctypes.c_double)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("prec", ctypes.c_int), ("in_dtype", ctypes.c_int),
                ("out_dtype", ctypes.c_int), ("max_batch", ctypes.c_int), ("max_inflight", ctypes.c_int),
                ("plan_threads", ctypes.c_int), ("batch", BatchOptions), ("dense_below", ctypes.c_int),
                ("dense_below_1d", ctypes.c_int)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("cold", ctypes.c_int), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double),
                ("plan_seconds", ctypes.c_double), ("status", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("plan_hits", ctypes.c_uint64), ("plan_misses", ctypes.c_uint64),
                ("plans_cached", ctypes.c_uint64), ("plans_evicted", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("coeffs", ctypes.c_double), ("arena_bytes", ctypes.c_size_t),
                ("arena_used", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t), ("queued", ctypes.c_int),
                ("admitted", ctypes.c_int), ("running", ctypes.c_int)]


_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)

# name -> (argtypes)
SYMBOLS = {
    "jt_plan": [ctypes.c_int, _ip, _dp, _dp, ctypes.c_double, ctypes.POINTER(_vp)],
    "jt_plan_ex": [ctypes.c_int, _ip, _dp, _dp, ctypes.c_double, ctypes.POINTER(PlanOptions),
                   ctypes.POINTER(_vp)],
    "jt_plan_points": [ctypes.c_int, _ip, _dp, _dp, _dp, ctypes.c_double, ctypes.POINTER(PlanOptions),
                       ctypes.POINTER(_vp)],
    "jt_plan_destroy": [_vp],
    "jt_plan_dims": [_vp, _ip],
    "jt_plan_info": [_vp, ctypes.c_int, ctypes.POINTER(AxisInfo)],
    "jt_plan_nodes": [_vp, ctypes.c_int, _dp, _dp, _dp],
    "jt_plan_factors": [_vp, ctypes.c_int, _i32p, _dp, _dp, _dp],
    "jt_plan_entries": [_vp, ctypes.c_int, ctypes.c_int, _ip, _ip, _dp],
    "jt_plan_device_bytes": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "jt_plan_bind": [_vp, _vp, ctypes.c_size_t, _vp],
    "jt_plan_pack": [_vp, _vp, ctypes.c_size_t],
    "jt_workspace_bytes": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "jt_forward": [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp],
    "jt_inverse": [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp],
    "jt_apply_axis": [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int,
                      _vp],
    "jt_plan_many": [ctypes.c_int, _ip, _ip, _dp, _dp, ctypes.c_double, ctypes.POINTER(PlanOptions), _vp],
    "jt_batch_create": [ctypes.c_int, _vp, _ip, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(BatchOptions), ctypes.POINTER(_vp)],
    "jt_batch_destroy": [_vp],
    "jt_batch_info_get": [_vp, ctypes.POINTER(BatchInfo)],
    "jt_batch_tables": [_vp, _i32p, _i32p],
    "jt_batch_device_bytes": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "jt_batch_bind": [_vp, _vp, ctypes.c_size_t, _vp],
    "jt_batch_run": [_vp, _vp, _vp, _vp],
    "jt_batch_run_static": [_vp, _vp, _vp, _vp],
    "jt_batch_capture": [_vp, _vp, _vp],
    "jt_batch_replay": [_vp, _vp],
    "jt_batch_errors": [_vp, _vp, ctypes.POINTER(ctypes.c_uint32)],
    "jt_server_create": [_vp, ctypes.c_size_t, ctypes.POINTER(ServerOptions), ctypes.POINTER(_vp)],
    "jt_server_submit": [_vp, ctypes.c_int, _ip, _dp, _dp, ctypes.c_int, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)],
    "jt_server_poll": [_vp, ctypes.c_uint64, ctypes.POINTER(RequestInfo)],
    "jt_server_wait": [_vp, ctypes.c_uint64, ctypes.POINTER(RequestInfo)],
    "jt_server_stats_get": [_vp, ctypes.POINTER(ServerStats)],
    "jt_server_destroy": [_vp],
}
for _name, _args in SYMBOLS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.jt_last_error.restype = ctypes.c_char_p
_lib.jt_last_error.argtypes = []
_lib.jt_version.restype = ctypes.c_int
_lib.jt_version.argtypes = []
_lib.jt_clock.restype = ctypes.c_double
_lib.jt_clock.argtypes = []


def clock() -> float:
    """The monotonic clock (seconds) the server stamps requests with."""
    return _lib.jt_clock()


class JTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


def _check(st: int) -> None:
    if st != JT_OK:
        raise JTError(st, _lib.jt_last_error().decode(errors="replace"))


def version() -> int:
    return _lib.jt_version()


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


class Plan:
    """A d-dimensional uniform Jacobi transform plan (d = 1, 2, 3).

    n: sizes per axis; ab: (a, b) per axis; tol: low-rank tolerance.
    """

    def __init__(self, n: Sequence[int], ab: Sequence[Sequence[float]], tol: float,
                 nu0: int = 0, dense_below: int = -1, oversample: int = 0, iterations: int = 0,
                 seed: int = 0, kind: int = 1, planner: int = 0):
        self.n = tuple(int(v) for v in n)
        self.ab = tuple((float(a), float(b)) for a, b in ab)
        if len(self.ab) != len(self.n):
            raise ValueError("need one (a, b) pair per axis")
        self.tol = float(tol)
        d = len(self.n)
        nn = (ctypes.c_int * d)(*self.n)
        aa = (ctypes.c_double * d)(*[p[0] for p in self.ab])
        bb = (ctypes.c_double * d)(*[p[1] for p in self.ab])
        opt = PlanOptions(nu0, dense_below, oversample, iterations, seed, kind, planner)
        h = _vp()
        _check(_lib.jt_plan_ex(d, nn, aa, bb, self.tol, ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self._dev = None

    @classmethod
    def at_points(cls, points, ab: Sequence[Sequence[float]], tol: float, nu0: int = 0, dense_below: int = -1,
                  oversample: int = 0, iterations: int = 0, seed: int = 0, kind: int = 1):
        """Plan of the nonuniform forward transform (jt_plan_points): points[i]
        holds axis i's angles in (0, pi), non-decreasing; that axis has as many
        coefficients as points.  Only forward() applies it."""
        pts = [np.ascontiguousarray(p, dtype=np.float64).ravel() for p in points]
        self = cls.__new__(cls)
        self.n = tuple(len(p) for p in pts)
        self.ab = tuple((float(a), float(b)) for a, b in ab)
        if len(self.ab) != len(self.n):
            raise ValueError("need one (a, b) pair per axis")
        self.tol = float(tol)
        d = len(self.n)
        flat = np.concatenate(pts) if pts else np.zeros(0)
        nn = (ctypes.c_int * d)(*self.n)
        aa = (ctypes.c_double * d)(*[p[0] for p in self.ab])
        bb = (ctypes.c_double * d)(*[p[1] for p in self.ab])
        opt = PlanOptions(nu0, dense_below, oversample, iterations, seed, kind)
        h = _vp()
        self._h = None
        self._dev = None
        _check(_lib.jt_plan_points(d, nn, _dptr(flat), aa, bb, self.tol, ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self.points = pts
        return self

    @classmethod
    def _adopt(cls, handle, n, ab, tol):
        """Wrap a plan handle built by the library (jt_plan_many)."""
        self = cls.__new__(cls)
        self.n = tuple(int(v) for v in n)
        self.ab = tuple((float(a), float(b)) for a, b in ab)
        self.tol = float(tol)
        self._h = _vp(handle)
        self._dev = None
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.jt_plan_destroy(h)
            self._h = None

    @property
    def d(self) -> int:
        return len(self.n)

    def info(self, axis: int) -> dict:
        inf = AxisInfo()
        _check(_lib.jt_plan_info(self._h, axis, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in AxisInfo._fields_}

    def nodes(self, axis: int):
        n = self.n[axis]
        t, x, w = np.empty(n), np.empty(n), np.empty(n)
        _check(_lib.jt_plan_nodes(self._h, axis, _dptr(t), _dptr(x), _dptr(w)))
        return t, x, w

    def factors(self, axis: int):
        """Host copies (bins, WV (nu0 x n), U (r x n complex), V (r x (n-nu0) complex))."""
        inf = self.info(axis)
        n, nu0, r = inf["n"], inf["nu0"], inf["rank"]
        bins = np.empty(n, dtype=np.int32)
        wv = np.empty(nu0 * n)
        u = np.empty(2 * r * n)
        v = np.empty(2 * r * (n - nu0))
        _check(_lib.jt_plan_factors(self._h, axis, bins.ctypes.data_as(_i32p), _dptr(wv), _dptr(u),
                                    _dptr(v)))
        U = u.view(np.complex128).reshape(r, n)
        V = v.view(np.complex128).reshape(r, n - nu0)
        return bins, wv.reshape(nu0, n), U, V

    def entries(self, axis: int, rows, degrees) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        degrees = np.ascontiguousarray(degrees, dtype=np.int32)
        out = np.empty(2 * len(rows))
        _check(_lib.jt_plan_entries(self._h, axis, len(rows), rows.ctypes.data_as(_ip),
                                    degrees.ctypes.data_as(_ip), _dptr(out)))
        return out.view(np.complex128)

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(_lib.jt_plan_device_bytes(self._h, ctypes.byref(b)))
        return b.value

    def pack(self) -> np.ndarray:
        """Host copy of the packed factor image that bind() places on the device."""
        out = np.empty(self.device_bytes(), dtype=np.uint8)
        _check(_lib.jt_plan_pack(self._h, _vp(out.ctypes.data), out.nbytes))
        return out

    # ------------------------------------------------------------ device side
    def bind(self, device=None, stream=None):
        """Allocate the factor buffer with torch on `device` and copy the factors in."""
        import torch

        device = torch.device(device or "cuda")
        nbytes = self.device_bytes()
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        self._dev = buf
        self._dev_off = off
        st = stream if stream is not None else torch.cuda.current_stream(device)
        _check(_lib.jt_plan_bind(self._h, _vp(buf.data_ptr() + off), nbytes, _vp(st.cuda_stream)))
        return self

    @staticmethod
    def _dtype_code(t) -> int:
        import torch

        if t.dtype == torch.float64:
            return F64
        if t.dtype == torch.float32:
            return F32
        raise TypeError("tensors must be float32 or float64")

    def _check_tensor(self, t):
        import torch

        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("expected a CUDA (HIP) torch tensor")
        if tuple(t.shape) != self.n or not t.is_contiguous():
            raise ValueError("expected a contiguous tensor of shape %r, got %r" % (self.n, tuple(t.shape)))

    def _run(self, fn, x, out, prec, stream):
        import torch

        if self._dev is None:
            raise JTError(JT_ESTATE, "plan is not bound; call bind()")
        self._check_tensor(x)
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=x.device)
        self._check_tensor(out)
        st = stream if stream is not None else torch.cuda.current_stream(x.device)
        _check(fn(self._h, _vp(x.data_ptr()), self._dtype_code(x), _vp(out.data_ptr()),
                  self._dtype_code(out), int(prec), _vp(st.cuda_stream)))
        return out

    def forward(self, alpha, out=None, prec: int = PREC_FP64, stream=None):
        """g = (W0 J0 (x) ...) alpha, on the GPU."""
        return self._run(_lib.jt_forward, alpha, out, prec, stream)

    def inverse(self, g, out=None, prec: int = PREC_FP64, stream=None):
        """alpha = (W0 J0 (x) ...)^T g, on the GPU."""
        return self._run(_lib.jt_inverse, g, out, prec, stream)

    def apply_axis(self, axis: int, direction: int, x, out=None, prec: int = PREC_FP64, stream=None):
        import torch

        if self._dev is None:
            raise JTError(JT_ESTATE, "plan is not bound; call bind()")
        self._check_tensor(x)
        if out is None:
            out = torch.empty(self.n, dtype=x.dtype, device=x.device)
        self._check_tensor(out)
        st = stream if stream is not None else torch.cuda.current_stream(x.device)
        _check(_lib.jt_apply_axis(self._h, axis, direction, _vp(x.data_ptr()), self._dtype_code(x),
                                  _vp(out.data_ptr()), self._dtype_code(out), int(prec),
                                  _vp(st.cuda_stream)))
        return out


# ---------------------------------------------------------------- many plans, batches
def plan_many(shapes, abs_, tol: float, dense_below=None, planner: int = 0):
    """Build one plan per item on the host, one host thread per plan.

    shapes: per item a tuple of sizes (d = 1..3); abs_: per item a tuple of (a, b)
    pairs; dense_below: None, or per item the dense-path threshold (the
    FFT-vs-direct crossover); planner: jt_plan_options.planner for every item."""
    count = len(shapes)
    dims = [len(s) for s in shapes]
    flat_n = [int(v) for s in shapes for v in s]
    flat_a = [float(p[0]) for ab in abs_ for p in ab]
    flat_b = [float(p[1]) for ab in abs_ for p in ab]
    if len(flat_a) != len(flat_n):
        raise ValueError("need one (a, b) pair per axis of every item")
    handles = (_vp * count)()
    opts = None
    if dense_below is not None or planner:
        arr = (PlanOptions * count)()
        for i in range(count):
            arr[i].dense_below = -1 if dense_below is None else int(dense_below[i])
            arr[i].planner = int(planner)
        opts = arr
    _check(_lib.jt_plan_many(count, (ctypes.c_int * count)(*dims), (ctypes.c_int * len(flat_n))(*flat_n),
                             (ctypes.c_double * len(flat_a))(*flat_a), (ctypes.c_double * len(flat_b))(*flat_b),
                             float(tol), opts, ctypes.cast(handles, _vp)))
    return [Plan._adopt(handles[i], shapes[i], abs_[i], tol) for i in range(count)]


class PlanArena:
    """One device buffer holding the bound factors of many plans."""

    def __init__(self, plans, device=None, stream=None):
        import torch

        device = torch.device(device or "cuda")
        offs, total = [], 0
        for p in plans:
            offs.append(total)
            total += (p.device_bytes() + 255) // 256 * 256
        self.buf = torch.empty(total + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr() + (-self.buf.data_ptr()) % 256
        st = stream if stream is not None else torch.cuda.current_stream(device)
        for p, o in zip(plans, offs):
            _check(_lib.jt_plan_bind(p._h, _vp(base + o), p.device_bytes(), _vp(st.cuda_stream)))
            p._dev = self.buf
        self.bytes = total


class Batch:
    """Many independent transforms in one persistent launch (jt_batch_*).

    plans: bound plans; dirs: FORWARD/INVERSE per item; in_offsets/out_offsets:
    element offsets of each item's tensor in the flat input/output buffers
    passed to run(); in_dtype/out_dtype: F64 or F32; prec: PREC_*."""

    def __init__(self, plans, dirs, in_offsets, out_offsets, in_dtype=F64, out_dtype=F64, prec=PREC_FP32_BULK,
                 max_split=0, min_units=0, grid=0):
        count = len(plans)
        self.plans = list(plans)  # keep the plans alive
        isz = 8 if in_dtype == F64 else 4
        osz = 8 if out_dtype == F64 else 4
        hs = (_vp * count)(*[p._h.value for p in plans])
        ioff = (ctypes.c_uint64 * count)(*[int(o) * isz for o in in_offsets])
        ooff = (ctypes.c_uint64 * count)(*[int(o) * osz for o in out_offsets])
        opt = BatchOptions(int(max_split), int(min_units), int(grid))
        h = _vp()
        _check(_lib.jt_batch_create(count, ctypes.cast(hs, _vp), (ctypes.c_int * count)(*[int(d) for d in dirs]),
                                    ioff, ooff, int(in_dtype), int(out_dtype), int(prec), ctypes.byref(opt),
                                    ctypes.byref(h)))
        self._h = h
        self._dev = None
        self.in_dtype, self.out_dtype = in_dtype, out_dtype

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.jt_batch_destroy(h)
            self._h = None

    def info(self) -> dict:
        inf = BatchInfo()
        _check(_lib.jt_batch_info_get(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in BatchInfo._fields_}

    def tables(self):
        """(units: (U, 7) int32 in queue order, passes: (P, 4) int32)."""
        inf = self.info()
        u = np.empty((inf["units"], 7), dtype=np.int32)
        p = np.empty((inf["passes"], 4), dtype=np.int32)
        _check(_lib.jt_batch_tables(self._h, u.ctypes.data_as(_i32p), p.ctypes.data_as(_i32p)))
        return u, p

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(_lib.jt_batch_device_bytes(self._h, ctypes.byref(b)))
        return b.value

    def bind(self, device=None, stream=None):
        import torch

        device = torch.device(device or "cuda")
        nbytes = self.device_bytes()
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        st = stream if stream is not None else torch.cuda.current_stream(device)
        _check(_lib.jt_batch_bind(self._h, _vp(buf.data_ptr() + off), nbytes, _vp(st.cuda_stream)))
        self._dev = buf
        return self

    def _bufs(self, inp, out):
        import torch

        want_in = torch.float64 if self.in_dtype == F64 else torch.float32
        want_out = torch.float64 if self.out_dtype == F64 else torch.float32
        if not (isinstance(inp, torch.Tensor) and inp.is_cuda and inp.dtype == want_in and inp.is_contiguous()):
            raise TypeError("input must be a contiguous CUDA tensor of dtype %s" % want_in)
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == want_out and out.is_contiguous()):
            raise TypeError("output must be a contiguous CUDA tensor of dtype %s" % want_out)
        return _vp(inp.data_ptr()), _vp(out.data_ptr())

    def run(self, inp, out, stream=None):
        import torch

        i, o = self._bufs(inp, out)
        st = stream if stream is not None else torch.cuda.current_stream(inp.device)
        _check(_lib.jt_batch_run(self._h, i, o, _vp(st.cuda_stream)))
        return out

    def run_static(self, inp, out, stream=None):
        """As run(), with the run's counters in the library's own device array
        (jt_batch_run_static: allocates nothing; runs on one device must not overlap)."""
        import torch

        i, o = self._bufs(inp, out)
        st = stream if stream is not None else torch.cuda.current_stream(inp.device)
        _check(_lib.jt_batch_run_static(self._h, i, o, _vp(st.cuda_stream)))
        return out

    def capture(self, inp, out):
        i, o = self._bufs(inp, out)
        self._graph_bufs = (inp, out)
        _check(_lib.jt_batch_capture(self._h, i, o))
        return self

    def replay(self, stream=None):
        import torch

        st = stream if stream is not None else torch.cuda.current_stream(self._graph_bufs[0].device)
        _check(_lib.jt_batch_replay(self._h, _vp(st.cuda_stream)))

    def errors(self, stream=None) -> int:
        import torch

        st = stream if stream is not None else torch.cuda.current_stream()
        v = ctypes.c_uint32()
        _check(_lib.jt_batch_errors(self._h, _vp(st.cuda_stream), ctypes.byref(v)))
        return v.value


# ---------------------------------------------------------------- serving
def _info_dict(inf: RequestInfo) -> dict:
    return {f: getattr(inf, f) for f, _ in RequestInfo._fields_}


class Server:
    """Continuous-batching request loop over a device arena (jt_server_*).

    arena_bytes of device memory are allocated with torch and handed to the
    server, which sub-allocates request buffers, cached axis plans and launch
    tables in it.  submit() takes host numpy arrays (pinned memory lets the
    copies overlap); the output array must stay alive until wait() returns."""

    def __init__(self, arena_bytes: int, tol: float = 1e-7, prec: int = PREC_FP32_BULK, dtype: int = F32,
                 max_batch: int = 0, max_inflight: int = 0, plan_threads: int = 0, device=None,
                 max_split: int = 0, min_units: int = 0, grid: int = 0, dense_below: int = 0,
                 dense_below_1d: int = 0):
        import torch

        device = torch.device(device or "cuda")
        self._arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=device)
        base = self._arena.data_ptr() + (-self._arena.data_ptr()) % 256
        torch.cuda.synchronize(device)
        opt = ServerOptions(float(tol), int(prec), int(dtype), int(dtype), int(max_batch), int(max_inflight),
                            int(plan_threads), BatchOptions(int(max_split), int(min_units), int(grid)),
                            int(dense_below), int(dense_below_1d))
        h = _vp()
        _check(_lib.jt_server_create(_vp(base), int(arena_bytes), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self.dtype = np.float64 if dtype == F64 else np.float32
        self._keep = {}

    def submit(self, x: np.ndarray, out: np.ndarray, ab, direction: int = FORWARD) -> int:
        x = np.asarray(x)
        if x.dtype != self.dtype or out.dtype != self.dtype or not x.flags.c_contiguous or not out.flags.c_contiguous:
            raise TypeError("input and output must be C-contiguous %s arrays" % np.dtype(self.dtype).name)
        if x.shape != out.shape:
            raise ValueError("input and output shapes differ")
        d = x.ndim
        if len(ab) != d:
            raise ValueError("need one (a, b) pair per axis")
        t = ctypes.c_uint64()
        _check(_lib.jt_server_submit(self._h, d, (ctypes.c_int * d)(*x.shape),
                                     (ctypes.c_double * d)(*[float(p[0]) for p in ab]),
                                     (ctypes.c_double * d)(*[float(p[1]) for p in ab]), int(direction),
                                     _vp(x.ctypes.data), _vp(out.ctypes.data), ctypes.byref(t)))
        self._keep[t.value] = (x, out)
        return t.value

    def poll(self, ticket: int) -> dict:
        inf = RequestInfo()
        _check(_lib.jt_server_poll(self._h, ticket, ctypes.byref(inf)))
        return _info_dict(inf)

    def wait(self, ticket: int) -> dict:
        inf = RequestInfo()
        st = _lib.jt_server_wait(self._h, ticket, ctypes.byref(inf))
        self._keep.pop(ticket, None)
        _check(st)
        return _info_dict(inf)

    def stats(self) -> dict:
        s = ServerStats()
        _check(_lib.jt_server_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.jt_server_destroy(h)
            self._h = None

    def __del__(self):
        self.close()
