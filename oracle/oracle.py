"""ctypes wrapper of the FP64 CPU oracle (``sic_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is the parity reference for the GPU
library.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use it; the product path never imports this module.

Every function takes the same arrays the GPU library takes (per-sheet tracer
counts, segment charges and closure flags; tracer positions and velocities
sheet after sheet) and returns NumPy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sic_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
ROW = 8  # step, t, W_E, KE, momentum, total_charge, max_segment, flags
COLS = ("step", "t", "W_E", "KE", "momentum", "total_charge", "max_segment", "flags")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with plain IEEE semantics (no FMA contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                        "-shared", "-o", tmp, SRC, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        P = ctypes.c_void_p
        L.orc_wrap.restype = d
        L.orc_wrap.argtypes = [d, d]
        L.orc_min_image.restype = d
        L.orc_min_image.argtypes = [d, d, d]
        L.orc_point_cell.restype = ctypes.c_int
        L.orc_point_cell.argtypes = [d, d, ctypes.c_int]
        L.orc_deposit_segment.restype = d
        L.orc_deposit_segment.argtypes = [d, d, d, d, ctypes.c_int, P]
        L.orc_deposit.restype = None
        L.orc_deposit.argtypes = [d, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
        L.orc_solve.restype = None
        L.orc_solve.argtypes = [d, ctypes.c_int, P, P, P, P]
        L.orc_gather.restype = d
        L.orc_gather.argtypes = [d, ctypes.c_int, P, d]
        L.orc_gather_many.restype = None
        L.orc_gather_many.argtypes = [d, ctypes.c_int, P, i64, P, P]
        L.orc_push.restype = None
        L.orc_push.argtypes = [d, ctypes.c_int, d, ctypes.c_int, P, P, P, P, P, P, P, P]
        L.orc_push_c.restype = None
        L.orc_push_c.argtypes = [d, ctypes.c_int, d, ctypes.c_int, P, P, P, P, P, P, P, P]
        L.orc_deposit_linear.restype = None
        L.orc_deposit_linear.argtypes = [d, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
        L.orc_deposit_cic.restype = None
        L.orc_deposit_cic.argtypes = [d, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
        for name in ("orc_deposit_c", "orc_deposit_linear_c", "orc_deposit_cic_c"):
            getattr(L, name).restype = None
            getattr(L, name).argtypes = [d, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
        L.orc_refine.restype = i64
        L.orc_refine.argtypes = [d, d, ctypes.c_int, P, P, P, P, P, i64]
        L.orc_run_seg.restype = ctypes.c_int
        L.orc_run_seg.argtypes = [ctypes.c_int, d, ctypes.c_int, d, ctypes.c_int, P, P, P, P, P, i64, ctypes.c_int,
                                  i64, d, i64, P, P, P, P, P, P]
        L.orc_run_order.restype = ctypes.c_int
        L.orc_run_order.argtypes = [ctypes.c_int, d, ctypes.c_int, d, ctypes.c_int, P, P, P, P, P, i64,
                                    ctypes.c_int, i64, P, P, P, P, P]
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [d, ctypes.c_int, d, ctypes.c_int, P, P, P, P, P, i64, ctypes.c_int, i64,
                              P, P, P, P, P]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def wrap(x: float, L: float) -> float:
    return lib().orc_wrap(float(x), float(L))


def min_image(a: float, b: float, L: float) -> float:
    return lib().orc_min_image(float(a), float(b), float(L))


def point_cell(x: float, L: float, nc: int) -> int:
    return lib().orc_point_cell(float(x), float(L), int(nc))


def deposit_segment(a: float, b: float, q: float, L: float, nc: int) -> np.ndarray:
    Q = np.zeros(nc)
    lib().orc_deposit_segment(float(a), float(b), float(q), float(L), int(nc), _p(Q))
    return Q


def uniform_charges(n_tracers, q, closed):
    """Per-segment charges of sheets whose segments all carry the sheet's
    charge: entry t belongs to the segment that starts at tracer t; the last
    tracer of an open sheet starts no segment and gets 0."""
    nt, cl = _i32(n_tracers), _i32(closed)
    c = np.repeat(_f64(q), nt)
    ends = np.cumsum(nt) - 1
    c[ends[cl == 0]] = 0.0
    return c


def deposit(L, nc, n_tracers, q, closed, x, order=0, c=None):
    """Charge per cell Q_j (dx * density, mean not removed) and the longest
    segment; order 0: piecewise-constant segments, 1: piecewise-linear,
    2: first-order (W_1) weighting of constant segments.  ``c`` (per-segment
    charges, one per tracer) replaces the per-sheet ``q`` when given."""
    nt, qq, cl, xx = _i32(n_tracers), _f64(q), _i32(closed), _f64(x)
    Q = np.zeros(int(nc))
    ms = ctypes.c_double(0.0)
    if c is None:
        fn = {0: lib().orc_deposit, 1: lib().orc_deposit_linear, 2: lib().orc_deposit_cic}[order]
        fn(float(L), int(nc), len(nt), _p(nt), _p(qq), _p(cl), _p(xx), _p(Q), ctypes.byref(ms))
    else:
        cc = _f64(c)
        fn = {0: lib().orc_deposit_c, 1: lib().orc_deposit_linear_c, 2: lib().orc_deposit_cic_c}[order]
        fn(float(L), int(nc), len(nt), _p(nt), _p(cl), _p(cc), _p(xx), _p(Q), ctypes.byref(ms))
    return Q, ms.value


def refine(L, l_max, n_tracers, closed, x, v, c):
    """One refinement pass; returns (n_tracers, x, v, c, inserted)."""
    nt, cl = _i32(n_tracers).copy(), _i32(closed)
    n = len(x)
    cap = 2 * n
    xx, vv, cc = np.zeros(cap), np.zeros(cap), np.zeros(cap)
    xx[:n], vv[:n], cc[:n] = _f64(x), _f64(v), _f64(c)
    added = lib().orc_refine(float(L), float(l_max), len(nt), _p(nt), _p(cl), _p(xx), _p(vv), _p(cc), cap)
    if added < 0:
        raise MemoryError("refinement failed")
    m = n + added
    return nt, xx[:m].copy(), vv[:m].copy(), cc[:m].copy(), int(added)


def solve(L, nc, Q):
    """Field at the cell centres, W_E and the total charge."""
    QQ = _f64(Q)
    E = np.zeros(int(nc))
    W = ctypes.c_double(0.0)
    qt = ctypes.c_double(0.0)
    lib().orc_solve(float(L), int(nc), _p(QQ), _p(E), ctypes.byref(W), ctypes.byref(qt))
    return E, W.value, qt.value


def gather(L, nc, E, x):
    EE, xx = _f64(E), _f64(np.atleast_1d(x))
    out = np.zeros(len(xx))
    lib().orc_gather_many(float(L), int(nc), _p(EE), len(xx), _p(xx), _p(out))
    return out


def push(L, nc, dt, n_tracers, q, closed, E, x, v, c=None):
    """One leapfrog move with field E; returns new (x, v), KE and momentum."""
    nt, qq, cl, EE = _i32(n_tracers), _f64(q), _i32(closed), _f64(E)
    xx, vv = _f64(x).copy(), _f64(v).copy()
    ke = ctypes.c_double(0.0)
    mom = ctypes.c_double(0.0)
    if c is None:
        lib().orc_push(float(L), int(nc), float(dt), len(nt), _p(nt), _p(qq), _p(cl), _p(EE), _p(xx), _p(vv),
                       ctypes.byref(ke), ctypes.byref(mom))
    else:
        cc = _f64(c)
        lib().orc_push_c(float(L), int(nc), float(dt), len(nt), _p(nt), _p(cl), _p(cc), _p(EE), _p(xx), _p(vv),
                         ctypes.byref(ke), ctypes.byref(mom))
    return xx, vv, ke.value, mom.value


def run(L, nc, dt, n_tracers, q, closed, x0, v0, n_steps, step0=0, init_kick=True, order=0):
    """Full run.  Returns dict(hist=[n_steps+1, 8], x, v (= v^{N-1/2}), Q, E)."""
    nt, qq, cl = _i32(n_tracers), _f64(q), _i32(closed)
    xx, vv = _f64(x0), _f64(v0)
    n = int(np.sum(nt, dtype=np.int64))
    if len(xx) != n or len(vv) != n:
        raise ValueError("x0/v0 length must equal the total tracer count")
    hist = np.zeros((int(n_steps) + 1, ROW))
    xo, vo = np.zeros(n), np.zeros(n)
    Qo, Eo = np.zeros(int(nc)), np.zeros(int(nc))
    rc = lib().orc_run_order(int(order), float(L), int(nc), float(dt), len(nt), _p(nt), _p(qq), _p(cl), _p(xx),
                             _p(vv), int(step0), 1 if init_kick else 0, int(n_steps), _p(hist), _p(xo), _p(vo),
                             _p(Qo), _p(Eo))
    if rc != 0:
        raise MemoryError("oracle run failed")
    return dict(hist=hist, x=xo, v=vo, Q=Qo, E=Eo)


def run_seg(L, nc, dt, n_tracers, closed, c, x0, v0, n_steps, step0=0, init_kick=True, order=0, l_max=0.0,
            capacity=None):
    """Full run with per-segment charges ``c`` and, when ``l_max`` > 0,
    refinement after every move.  Returns dict(hist, count (tracers after
    each step), n_tracers, c, x, v, Q, E)."""
    nt, cl = _i32(n_tracers).copy(), _i32(closed)
    cc = _f64(c).copy()
    xx, vv = _f64(x0), _f64(v0)
    n = int(np.sum(nt, dtype=np.int64))
    if len(xx) != n or len(vv) != n or len(cc) != n:
        raise ValueError("x0/v0/c length must equal the total tracer count")
    cap = n if capacity is None else max(int(capacity), n)
    cbuf = np.zeros(cap)
    cbuf[:n] = cc
    hist = np.zeros((int(n_steps) + 1, ROW))
    count = np.zeros(int(n_steps) + 1, dtype=np.int64)
    xo, vo = np.zeros(cap), np.zeros(cap)
    Qo, Eo = np.zeros(int(nc)), np.zeros(int(nc))
    rc = lib().orc_run_seg(int(order), float(L), int(nc), float(dt), len(nt), _p(nt), _p(cl), _p(cbuf), _p(xx),
                           _p(vv), int(step0), 1 if init_kick else 0, int(n_steps), float(l_max), cap, _p(hist),
                           _p(count), _p(xo), _p(vo), _p(Qo), _p(Eo))
    if rc == 1:
        raise MemoryError("oracle run failed")
    if rc == 2:
        raise MemoryError("refinement exceeded the tracer capacity")
    m = int(np.sum(nt, dtype=np.int64))
    return dict(hist=hist, count=count, n_tracers=nt, c=cbuf[:m].copy(), x=xo[:m].copy(), v=vo[:m].copy(), Q=Qo,
                E=Eo)


def run_problem(problem, n_steps=None, order=0):
    """Run an ``inputs.Problem`` for ``n_steps`` (default: its own step count)."""
    steps = problem.n_steps if n_steps is None else n_steps
    return run(problem.L, problem.n_cells, problem.dt, problem.n_tracers, problem.q, problem.closed,
               problem.x0, problem.v0, steps, order=order)
