"""CPU oracle for time-vectorized backward- and forward-Euler integration.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the HIP library in ``paper_2310_08649_amd`` and never imports it.

Contents
--------
* ``forward`` / ``adjoint``: ctypes front end of ``oracle.c``, the plain
  sequential backward-Euler integrator with a dense Newton solve per step
  (Section 2.2, Eq. backward-euler) and its discrete adjoint (Appendix A);
  with ``scheme="forward_euler"`` the explicit recurrence of Eq. forward-euler
  and the discrete adjoint of that map.
* ``rhs`` / ``vjp_p``: the model right-hand sides, their state Jacobians and
  parameter vector-Jacobian products, as the C oracle evaluates them.
* ``blockbidiag``: the plain definitions of the batched block-bidiagonal
  solves of Section 3 (dense assembly + ``numpy.linalg.solve``, and Thomas's
  algorithm, Alg. thomas).
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

from . import blockbidiag  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KINDS = {"linear": 0, "vanderpol": 1, "robertson": 2, "mlp": 3, "chaboche": 4, "neuron": 5, "mds": 6, "fnode": 7}
STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "SINGULAR", 3: "NONFINITE"}

_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "oracle.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm", "-lpthread"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.oracle_param_count.argtypes = [i32, i32, i32]
    lib.oracle_param_count.restype = i32
    lib.oracle_lu_solve.argtypes = [i32, P, P]
    lib.oracle_lu_solve.restype = i32
    lib.oracle_rhs.argtypes = [i32, i32, i32, P, f64, P, P, P]
    lib.oracle_rhs.restype = i32
    lib.oracle_vjp_p.argtypes = [i32, i32, i32, P, f64, P, P, P]
    lib.oracle_vjp_p.restype = i32
    lib.oracle_forward.argtypes = [i32, i32, i32, i64, i64, P, P, P, P, i32, f64, f64, i32, i32, P, P, P]
    lib.oracle_forward.restype = i32
    lib.oracle_adjoint.argtypes = [i32, i32, i32, i64, i64, P, P, P, P, i32, P, i32, P, P, P]
    lib.oracle_adjoint.restype = i32
    lib.oracle_forward_euler.argtypes = [i32, i32, i32, i64, i64, P, P, P, P, i32, i32, P, P]
    lib.oracle_forward_euler.restype = i32
    lib.oracle_forward_euler_adjoint.argtypes = [i32, i32, i32, i64, i64, P, P, P, P, i32, P, i32, P, P, P]
    lib.oracle_forward_euler_adjoint.restype = i32
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


@contextlib.contextmanager
def using_library(path):
    """Run the wrappers against another build of ``oracle.c`` (used by the
    tests that plant mistakes in a copy of the oracle to show the pins catch them)."""
    global _lib
    saved = _load()
    _lib = _bind(ctypes.CDLL(os.path.abspath(path)))
    try:
        yield
    finally:
        _lib = saved


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _kind(kind):
    return KINDS[kind] if isinstance(kind, str) else int(kind)


def param_count(kind, n, hidden=64):
    return _load().oracle_param_count(_kind(kind), n, hidden)


def default_threads():
    return max(1, len(os.sched_getaffinity(0)))


def lu_solve(A, b):
    """x with A x = b by LU with partial pivoting; raises on a singular pivot."""
    A = _f64(A).copy()
    x = _f64(b).copy()
    if _load().oracle_lu_solve(A.shape[0], _p(A), _p(x)):
        raise np.linalg.LinAlgError("singular pivot")
    return x


def rhs(kind, y, t, p, hidden=64):
    """(f, J): the model rate h(y,t;p) and its state Jacobian dh/dy."""
    y, p = _f64(y), _f64(p)
    n = y.shape[0]
    f = np.empty(n)
    J = np.empty((n, n))
    if _load().oracle_rhs(_kind(kind), n, hidden, _p(y), float(t), _p(p), _p(f), _p(J)):
        raise ValueError("bad model arguments")
    return f, J


def vjp_p(kind, y, t, p, w, hidden=64):
    """(dh/dp)^T w."""
    y, p, w = _f64(y), _f64(p), _f64(w)
    gp = np.zeros(p.shape[0])
    if _load().oracle_vjp_p(_kind(kind), y.shape[0], hidden, _p(y), float(t), _p(p), _p(w), _p(gp)):
        raise ValueError("bad model arguments")
    return gp


def _layout(y0, times, offsets):
    B, n = y0.shape
    if offsets is None:
        N = times.shape[0] - 1
        return B, n, N, None, (B, N + 1, n)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    if offsets.shape != (B + 1,) or offsets[0] != 0 or times.shape[0] != offsets[-1]:
        raise ValueError("offsets must be point offsets [B+1] starting at 0 and ending at len(times)")
    N = int(np.max(np.diff(offsets)) - 1) if B else 0
    return B, n, N, offsets, (int(offsets[-1]), n)


SCHEMES = ("backward_euler", "forward_euler")


def forward(kind, y0, times, params, offsets=None, tol=(1e-8, 1e-6), max_newton=50,
            threads=None, hidden=64, params_shared=None, scheme="backward_euler"):
    """Sequential backward Euler (dense Newton per step), or forward Euler
    (``scheme="forward_euler"``: no iteration, ``tol`` and ``max_newton`` unused,
    ``iters`` all zero).

    Returns ``(y, status, iters)`` with ``y`` in the layout of ``times``:
    ``[B, N+1, n]`` for a shared uniform grid, ``[points, n]`` for ragged
    series given by point ``offsets``.
    """
    if scheme not in SCHEMES:
        raise ValueError("scheme must be one of %s" % (SCHEMES,))
    y0, times, params = _f64(y0), _f64(times), _f64(params)
    B, n, N, offsets, shape = _layout(y0, times, offsets)
    if params_shared is None:
        params_shared = params.ndim == 1
    y = np.empty(shape)
    status = np.zeros(B, dtype=np.int32)
    iters = np.zeros(B, dtype=np.int32)
    if scheme == "forward_euler":
        rc = _load().oracle_forward_euler(
            _kind(kind), n, hidden, B, N, _p(offsets), _p(times), _p(y0), _p(params), int(params_shared),
            int(threads or default_threads()), _p(y), _p(status))
    else:
        rc = _load().oracle_forward(
            _kind(kind), n, hidden, B, N, _p(offsets), _p(times), _p(y0), _p(params), int(params_shared),
            float(tol[0]), float(tol[1]), int(max_newton), int(threads or default_threads()),
            _p(y), _p(status), _p(iters))
    if rc:
        raise ValueError("oracle_forward rejected its arguments (%d)" % rc)
    return y, status, iters


def adjoint(kind, y, times, params, g, offsets=None, threads=None, hidden=64, params_shared=None,
            scheme="backward_euler"):
    """Discrete adjoint of ``forward`` (same ``scheme``): returns ``(dLdp, dLdy0, status)``."""
    if scheme not in SCHEMES:
        raise ValueError("scheme must be one of %s" % (SCHEMES,))
    y, times, params, g = _f64(y), _f64(times), _f64(params), _f64(g)
    if offsets is None:
        B, n = y.shape[0], y.shape[2]
        y0 = y[:, 0, :]
    else:
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        B, n = offsets.shape[0] - 1, y.shape[1]
        y0 = y[offsets[:-1]]
    B, n, N, offsets, shape = _layout(np.empty((B, n)), times, offsets)
    if y.shape != shape or g.shape != shape:
        raise ValueError("y and g must have the trajectory layout %s" % (shape,))
    if params_shared is None:
        params_shared = params.ndim == 1
    P = param_count(kind, n, hidden)
    dLdp = np.zeros(P if params_shared else (B, P))
    dLdy0 = np.zeros((B, n))
    status = np.zeros(B, dtype=np.int32)
    fn = _load().oracle_forward_euler_adjoint if scheme == "forward_euler" else _load().oracle_adjoint
    rc = fn(_kind(kind), n, hidden, B, N, _p(offsets), _p(times), _p(y), _p(params), int(params_shared),
            _p(g), int(threads or default_threads()), _p(dLdp), _p(dLdy0), _p(status))
    if rc:
        raise ValueError("oracle_adjoint rejected its arguments (%d)" % rc)
    del y0
    return dLdp, dLdy0, status
