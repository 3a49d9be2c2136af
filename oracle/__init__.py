"""Oracle for the uniform multi-dimensional Jacobi transform.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
(C ABI + HIP kernels + its Python binding) never imports, links or calls it,
and this package imports nothing from the product.

What it computes (Section 3.1, eqs. (35)-(39); Section 3.2 eqs. (53)-(55);
Section 3.3 eqs. (56)-(60)):

* 1D:  A[j, k] = sqrt(omega_j) * phat_k(x_j), nodes ascending in t = arccos x,
  built by the C routine in ``jacobi_oracle.c`` (long-double internals).
  forward  g = A alpha,  inverse  alpha = A^T g  (A is orthogonal, Sec. 3.1).
* dD:  the Kronecker product of the per-axis matrices: axis i of a row-major
  tensor uses (n_i, a_i, b_i); forward applies A_i along every axis, inverse
  applies A_i^T along every axis (eqs. (54), (55), (59), (60)).

The apply step is a plain matrix product along each axis (numpy, fp64), with
no blocking, reordering or fusion beyond that.

Two more routines of the same C file serve checks the long-double build is
too slow for, and the nonuniform transform:

* ``apply1d_fp64`` / ``nodes_fp64``: the same 1D definition in plain fp64
  (nodes isolated by sign changes of phat_n on a grid in t and refined by
  safeguarded Newton; Christoffel weights; the sums by the recurrence, no
  matrix stored).  For checking fp32-bulk results of long 1D items.
* ``ptilde`` / ``forward_points``: the modified Jacobi functions
  Ptilde_k(t) = phat_k(cos t) sqrt(w(cos t) sin t) at given angles, and the
  nonuniform forward transform f = (P0 (x) P1 (x) ...) alpha with
  P_i[j, k] = Ptilde_k(t_{i,j}) (Section 3.1, the nonuniform remark after
  eq. (39); Sections 3.2-3.3 for 2D/3D), no quadrature weights.
* ``qtilde`` / ``matrix_q`` / ``forward_q`` / ``forward_points_q``: the
  modified Jacobi functions of the second kind (Section 1),
  Qtilde_k(t) = sqrt(sin t / w(x)) q_k(x) / pi with q_k the finite Hilbert
  transform of w phat_k (q_0 from Tricomi's closed form, then the
  inhomogeneous three-term recurrence), and the second-kind transforms: the
  uniform one with matrix sqrt(w_j) Qtilde_k(t_j) at the Gauss-Jacobi nodes
  and the nonuniform one at given angles (Section 3: "the transform for
  Qtilde is similar").  Parameters with exactly one of a, b equal to 0 are
  not supported by the closed form (ValueError).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libjacobi_oracle.so")
_lib = None
_cache: dict = {}


def build(force: bool = True) -> str:
    """Compile the oracle's C part (gcc, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_build.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        lib.orc_build.restype = ctypes.c_int
        lib.orc_recurrence.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        lib.orc_recurrence.restype = ctypes.c_int
        lib.orc_ptilde.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
        lib.orc_ptilde.restype = ctypes.c_int
        lib.orc_nodes_fp64.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.orc_nodes_fp64.restype = ctypes.c_int
        lib.orc_apply_fp64.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
        lib.orc_apply_fp64.restype = ctypes.c_int
        lib.orc_qtilde.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
        lib.orc_qtilde.restype = ctypes.c_int
        lib.orc_build_q.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_build_q.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def matrix(n: int, a: float, b: float):
    """Return (A, x, omega) for one axis; A is n x n row-major fp64, x descending."""
    key = (int(n), float(a), float(b))
    if key not in _cache:
        lib = _load()
        A = np.empty((n, n), dtype=np.float64)
        x = np.empty(n, dtype=np.float64)
        w = np.empty(n, dtype=np.float64)
        rc = lib.orc_build(int(n), float(a), float(b), _ptr(A), _ptr(x), _ptr(w))
        if rc != 0:
            raise ValueError("oracle: invalid parameters n=%r a=%r b=%r" % (n, a, b))
        _cache[key] = (A, x, w)
    return _cache[key]


def recurrence(n: int, a: float, b: float):
    """Recurrence coefficients (alpha_0..alpha_n, beta_0..beta_n, mu0) of the oracle."""
    lib = _load()
    al = np.empty(n + 1)
    be = np.empty(n + 1)
    mu = np.empty(1)
    rc = lib.orc_recurrence(int(n), float(a), float(b), _ptr(al), _ptr(be), _ptr(mu))
    if rc != 0:
        raise ValueError("oracle: invalid parameters")
    return al, be, float(mu[0])


def clear_cache() -> None:
    _cache.clear()
    _qcache.clear()


def _apply(x: np.ndarray, params, transpose: bool) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != len(params):
        raise ValueError("need one (a, b) pair per axis")
    for axis, (a, b) in enumerate(params):
        A = matrix(x.shape[axis], a, b)[0]
        M = A.T if transpose else A
        x = np.moveaxis(np.tensordot(M, x, axes=([1], [axis])), 0, axis)
    return np.ascontiguousarray(x)


def forward(alpha: np.ndarray, params) -> np.ndarray:
    """g = (A_0 (x) A_1 (x) ...) alpha for a row-major tensor alpha."""
    return _apply(alpha, params, transpose=False)


def inverse(g: np.ndarray, params) -> np.ndarray:
    """alpha = (A_0 (x) A_1 (x) ...)^T g."""
    return _apply(g, params, transpose=True)


def forward_entries(alpha: np.ndarray, params, index: np.ndarray) -> np.ndarray:
    """Entries g[index[s]] of the forward transform, each computed on its own.

    index: (S, d) integer array of output multi-indices.
    """
    return _entries(alpha, params, index, transpose=False)


def inverse_entries(g: np.ndarray, params, index: np.ndarray) -> np.ndarray:
    return _entries(g, params, index, transpose=True)


def _entries(x, params, index, transpose):
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    mats = []
    for axis, (a, b) in enumerate(params):
        A = matrix(x.shape[axis], a, b)[0]
        mats.append(A.T if transpose else A)
    out = np.empty(len(index))
    for s, idx in enumerate(np.asarray(index)):
        t = x
        # contract the last axis first with the needed row of its matrix
        for axis in range(d - 1, -1, -1):
            t = t @ mats[axis][idx[axis]]
        out[s] = t
    return out


# ------------------------------------------------------------------ plain fp64 1D path
def nodes_fp64(n: int, a: float, b: float):
    """(x, omega) in fp64: nodes descending in x (ascending in t), Christoffel weights."""
    x = np.empty(n)
    w = np.empty(n)
    rc = _load().orc_nodes_fp64(int(n), float(a), float(b), _ptr(x), _ptr(w))
    if rc != 0:
        raise ValueError("oracle: node search failed (code %d) for n=%r a=%r b=%r" % (rc, n, a, b))
    return x, w


def apply1d_fp64(v: np.ndarray, ab, transpose: bool = False) -> np.ndarray:
    """A v (transpose=False) or A^T v for one 1D axis, in plain fp64."""
    v = np.ascontiguousarray(v, dtype=np.float64).ravel()
    y = np.empty_like(v)
    rc = _load().orc_apply_fp64(len(v), float(ab[0]), float(ab[1]), 1 if transpose else 0, _ptr(v), _ptr(y))
    if rc != 0:
        raise ValueError("oracle: fp64 apply failed (code %d)" % rc)
    return y


# ------------------------------------------------------------------ nonuniform transform
def ptilde(n: int, a: float, b: float, t) -> np.ndarray:
    """P[j, k] = Ptilde_k(t_j) for k < n at the given angles t_j in (0, pi)."""
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    out = np.empty((len(t), n))
    rc = _load().orc_ptilde(int(n), float(a), float(b), len(t), _ptr(t), _ptr(out))
    if rc != 0:
        raise ValueError("oracle: bad arguments to ptilde (code %d)" % rc)
    return out


def forward_points(alpha: np.ndarray, params, points) -> np.ndarray:
    """Nonuniform forward transform: along axis i apply P_i[j, k] = Ptilde_k(t_{i,j})
    (points[i] = the angles of axis i); no quadrature weights."""
    x = np.asarray(alpha, dtype=np.float64)
    if x.ndim != len(params) or len(points) != x.ndim:
        raise ValueError("need one (a, b) pair and one point set per axis")
    for axis, ((a, b), t) in enumerate(zip(params, points)):
        P = ptilde(x.shape[axis], a, b, t)
        x = np.moveaxis(np.tensordot(P, x, axes=([1], [axis])), 0, axis)
    return np.ascontiguousarray(x)


# ------------------------------------------------------------------ second kind
def qtilde(n: int, a: float, b: float, t) -> np.ndarray:
    """Q[j, k] = Qtilde_k(t_j) for k < n at the given angles t_j in (0, pi)."""
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    out = np.empty((len(t), n))
    rc = _load().orc_qtilde(int(n), float(a), float(b), len(t), _ptr(t), _ptr(out))
    if rc != 0:
        raise ValueError("oracle: qtilde unsupported or bad arguments (code %d) for a=%r b=%r" % (rc, a, b))
    return out


_qcache = {}


def matrix_q(n: int, a: float, b: float) -> np.ndarray:
    """The uniform second-kind matrix Q[j, k] = sqrt(w_j) Qtilde_k(t_j) at the
    Gauss-Jacobi nodes (ascending t), w_j the trigonometric weights."""
    key = (int(n), float(a), float(b))
    if key not in _qcache:
        Q = np.empty((n, n))
        rc = _load().orc_build_q(int(n), float(a), float(b), _ptr(Q))
        if rc != 0:
            raise ValueError("oracle: second-kind matrix unsupported or bad arguments (code %d)" % rc)
        _qcache[key] = Q
    return _qcache[key]


def forward_q(alpha: np.ndarray, params) -> np.ndarray:
    """Uniform second-kind forward transform: Q_i along each axis i."""
    x = np.asarray(alpha, dtype=np.float64)
    if x.ndim != len(params):
        raise ValueError("need one (a, b) pair per axis")
    for axis, (a, b) in enumerate(params):
        Q = matrix_q(x.shape[axis], a, b)
        x = np.moveaxis(np.tensordot(Q, x, axes=([1], [axis])), 0, axis)
    return np.ascontiguousarray(x)


def forward_points_q(alpha: np.ndarray, params, points) -> np.ndarray:
    """Nonuniform second-kind forward transform: along axis i apply
    Q_i[j, k] = Qtilde_k(t_{i,j}); no quadrature weights."""
    x = np.asarray(alpha, dtype=np.float64)
    if x.ndim != len(params) or len(points) != x.ndim:
        raise ValueError("need one (a, b) pair and one point set per axis")
    for axis, ((a, b), t) in enumerate(zip(params, points)):
        Q = qtilde(x.shape[axis], a, b, t)
        x = np.moveaxis(np.tensordot(Q, x, axes=([1], [axis])), 0, axis)
    return np.ascontiguousarray(x)
