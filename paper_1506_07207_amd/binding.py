"""Python binding of libsic (argument marshalling only).

Every function here has the name of the C entry point it calls (include/sic.h)
and does no arithmetic of the method: all of the step runs in the HIP
kernels behind the C ABI.  Arrays may be NumPy arrays (host memory) or torch
tensors (host or CUDA/HIP device memory); device tensors are passed as device
pointers, so nothing crosses PCIe.

Importing this module does not load the library; the first call does, and
raises ``SicError`` if ``libsic.so`` has not been built (there is no fallback
path).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsic.so")

SIC_ABI_VERSION = 2
SIC_BATCH_SEGMENT_CHARGES = 1
SIC_MAX_CELLS = 4096
SIC_NOALLOC_MAX_TRACERS = 1 << 20
SIC_FP64, SIC_SPLIT_F32, SIC_SPLIT_U32 = 0, 1, 2
SIC_MEM_HOST, SIC_MEM_DEVICE = 0, 1
SIC_DIAG_NONFINITE, SIC_DIAG_LONG_SEGMENT = 1, 2
SIC_PATH_NONE, SIC_PATH_FUSED, SIC_PATH_RESIDENT, SIC_PATH_REFINING, SIC_PATH_SOLVE_FIRST = -1, 0, 1, 2, 3
STATUS = {0: "SIC_OK", 1: "SIC_EINVAL", 2: "SIC_ENOMEM", 3: "SIC_EDEVICE", 4: "SIC_ESTATE", 5: "SIC_EBUSY",
          6: "SIC_ENOTSUP"}
PRECISIONS = {"fp64": SIC_FP64, "split_f32": SIC_SPLIT_F32, "split_u32": SIC_SPLIT_U32}

DIAG_DTYPE = np.dtype([("step", "<i8"), ("t", "<f8"), ("W_E", "<f8"), ("KE", "<f8"), ("momentum", "<f8"),
                       ("total_charge", "<f8"), ("max_segment", "<f8"), ("flags", "<i8")])


class SicError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}" + (f" ({msg})" if msg else ""))


class sic_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("n_cells", ctypes.c_int32), ("L", ctypes.c_double),
                ("dt", ctypes.c_double), ("precision", ctypes.c_int32), ("deposit_order", ctypes.c_int32),
                ("history_rows", ctypes.c_int64), ("l_max", ctypes.c_double), ("max_tracers", ctypes.c_int64)]


class sic_sheet(ctypes.Structure):
    _fields_ = [("n_tracers", ctypes.c_int32), ("closed", ctypes.c_int32), ("q_seg", ctypes.c_double)]


class sic_diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64 if n in ("step", "flags") else ctypes.c_double) for n in DIAG_DTYPE.names]


class sic_tuning(ctypes.Structure):
    _fields_ = [("tile_chunks", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("fused_only", ctypes.c_int32)]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SIGS = {
    "sic_abi_version": (_I32, []),
    "sic_status_str": (ctypes.c_char_p, [_I32]),
    "sic_init": (_I32, [_P, _P, _I32, _P, _P, _P, _I32, _P, _P]),
    "sic_refine": (_I32, [_P, ctypes.c_double, _P]),
    "sic_get_layout": (_I32, [_P, _P, _P]),
    "sic_get_charges": (_I32, [_P, _P, _I32]),
    "sic_load_state": (_I32, [_P, _I64, _P, _P, _P, _P, _I32]),
    "sic_deposit": (_I32, [_P]),
    "sic_solve_field": (_I32, [_P]),
    "sic_push": (_I32, [_P]),
    "sic_step": (_I32, [_P, _I64]),
    "sic_diagnostics": (_I32, [_P, _P, _P, _P, _P, _P]),
    "sic_get_state": (_I32, [_P, _P, _P, _P, _I32]),
    "sic_set_state": (_I32, [_P, _I64, _P, _P, _I32]),
    "sic_set_state_noalloc": (_I32, [_P, _I64, _P, _P, _I32]),
    "sic_destroy": (None, [_P]),
    "sic_last_error": (ctypes.c_char_p, [_P]),
    "sic_set_tuning": (_I32, [_P, _P]),
    "sic_get_tuning": (_I32, [_P, _P]),
    "sic_set_timing": (_I32, [_P, _I32]),
    "sic_last_timing": (_I32, [_P, _P, _P]),
    "sic_last_step_path": (_I32, [_P, _P]),
    "sic_batch_create": (_I32, [_I64, _I32, _I32, _I32, _I32, _I32, _I64, _P, _P]),
    "sic_batch_admit": (_I32, [_P, _P, _P, _I32, _P, _P, _P, _I32, _I64, _P]),
    "sic_batch_get_charges": (_I32, [_P, _I32, _P, _I32]),
    "sic_batch_get_layout": (_I32, [_P, _I32, _P, _P]),
    "sic_batch_step": (_I32, [_P, _I64]),
    "sic_batch_poll": (_I32, [_P, _P, _I32, _P]),
    "sic_batch_result": (_I32, [_P, _I32, _P, _P, _P, _P, _P]),
    "sic_batch_get_state": (_I32, [_P, _I32, _P, _P, _P, _I32]),
    "sic_batch_release": (_I32, [_P, _I32]),
    "sic_batch_usage": (_I32, [_P, _P, _P]),
    "sic_batch_set_tuning": (_I32, [_P, _P]),
    "sic_batch_get_tuning": (_I32, [_P, _P]),
    "sic_batch_destroy": (None, [_P]),
    "sic_batch_last_error": (ctypes.c_char_p, [_P]),
    "sic_batch_set_timing": (_I32, [_P, _I32]),
    "sic_batch_last_timing": (_I32, [_P, _P, _P]),
    "sic_copy_bandwidth": (_I32, [_I64, _I32, _P, _P]),
    "sic_autotune": (_I32, [_P, _I32, _P, _P]),
    "sic_batch_autotune": (_I32, [_P, _I32, _P, _P]),
}


def load():
    """Loads libsic.so (raises SicError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SicError(2, "load", f"{LIB_PATH} is not built; run python -m paper_1506_07207_amd.build")
        # torch loads its own HIP runtime (same soname as the one libsic links
        # against).  Loading torch first makes libsic bind to that runtime, so
        # torch streams and device pointers are valid handles for libsic and
        # the process holds a single HIP runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def lib_path() -> str:
    return LIB_PATH


# ------------------------------------------------------------------ marshalling

def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch

            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _as_f64(a):
    """(pointer, mem_kind, keepalive) for a float64 array or tensor."""
    try:
        import torch

        if isinstance(a, torch.Tensor):
            if a.dtype != torch.float64:
                raise TypeError("tensor must be float64")
            t = a.contiguous()
            kind = SIC_MEM_DEVICE if t.is_cuda else SIC_MEM_HOST
            return ctypes.c_void_p(t.data_ptr()), kind, t
    except ImportError:
        pass
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return arr.ctypes.data_as(ctypes.c_void_p), SIC_MEM_HOST, arr


def _check(rc: int, where: str, handle=None, batch=False):
    if rc != 0:
        msg = ""
        try:
            fn = load().sic_batch_last_error if batch else load().sic_last_error
            msg = (fn(handle) or b"").decode()
        except Exception:
            pass
        raise SicError(rc, where, msg)


def make_config(L, n_cells, dt, precision=SIC_FP64, history_rows=0, deposit_order=0, l_max=0.0,
                max_tracers=0) -> sic_config:
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    return sic_config(SIC_ABI_VERSION, int(n_cells), float(L), float(dt), int(precision), int(deposit_order),
                      int(history_rows), float(l_max), int(max_tracers))


def make_sheets(n_tracers, q, closed=None):
    n = len(n_tracers)
    arr = (sic_sheet * n)()
    for i in range(n):
        arr[i].n_tracers = int(n_tracers[i])
        arr[i].closed = 1 if closed is None else int(closed[i])
        arr[i].q_seg = float(q[i])
    return arr


def _diag_dict(d: sic_diag) -> dict:
    return {n: getattr(d, n) for n in DIAG_DTYPE.names}


# ------------------------------------------------------------------ single simulation

def sic_abi_version() -> int:
    return load().sic_abi_version()


def sic_status_str(s: int) -> str:
    return load().sic_status_str(int(s)).decode()


def sic_init(L, n_cells, dt, n_tracers, q, closed, x0, v0, precision=SIC_FP64, history_rows=0, stream=None,
             deposit_order=0, seg_charges=None, l_max=0.0, max_tracers=0):
    """Creates a simulation (see sic_init in include/sic.h); returns the handle."""
    lib = load()
    cfg = make_config(L, n_cells, dt, precision, history_rows, deposit_order, l_max, max_tracers)
    sheets = make_sheets(n_tracers, q, closed)
    px, kx, kx_ = _as_f64(x0)
    pv, kv, kv_ = _as_f64(v0)
    pc, kc, kc_ = _as_f64(seg_charges) if seg_charges is not None else (None, kx, None)
    if kx != kv or kx != kc:
        raise ValueError("x0, v0 and seg_charges must live in the same memory")
    h = ctypes.c_void_p()
    rc = lib.sic_init(ctypes.byref(cfg), sheets, len(sheets), px, pv, pc, kx, _stream_ptr(stream), ctypes.byref(h))
    _check(rc, "sic_init")
    return h


def sic_deposit(h):
    _check(load().sic_deposit(h), "sic_deposit", h)


def sic_solve_field(h):
    _check(load().sic_solve_field(h), "sic_solve_field", h)


def sic_push(h):
    _check(load().sic_push(h), "sic_push", h)


def sic_step(h, n_steps: int):
    _check(load().sic_step(h, int(n_steps)), "sic_step", h)


def sic_diagnostics(h, n_cells: Optional[int] = None, history: bool = True):
    """Returns dict(last=row, rho=array|None, E=array|None, history=structured array|None)."""
    lib = load()
    last = sic_diag()
    rho = E = None
    prho = pE = None
    if n_cells:
        rho = np.zeros(int(n_cells))
        E = np.zeros(int(n_cells))
        prho = rho.ctypes.data_as(ctypes.c_void_p)
        pE = E.ctypes.data_as(ctypes.c_void_p)
    hist = None
    if history:
        n = ctypes.c_int64(0)
        _check(lib.sic_diagnostics(h, None, None, None, None, ctypes.byref(n)), "sic_diagnostics", h)
        hist = np.zeros(n.value, dtype=DIAG_DTYPE)
        _check(lib.sic_diagnostics(h, ctypes.byref(last), prho, pE, hist.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.byref(n)), "sic_diagnostics", h)
        hist = hist[: n.value]
    else:
        _check(lib.sic_diagnostics(h, ctypes.byref(last), prho, pE, None, None), "sic_diagnostics", h)
    return dict(last=_diag_dict(last), rho=rho, E=E, history=hist)


def sic_get_state(h, n_tracers_total: int, out_x=None, out_v=None):
    """Returns (x, v_half, step).  out_x/out_v may be device tensors."""
    lib = load()
    if out_x is None:
        out_x = np.zeros(int(n_tracers_total))
        out_v = np.zeros(int(n_tracers_total))
    px, kx, _ = _as_f64(out_x)
    pv, kv, _ = _as_f64(out_v)
    step = ctypes.c_int64(0)
    _check(lib.sic_get_state(h, px, pv, ctypes.byref(step), kx), "sic_get_state", h)
    return out_x, out_v, step.value


def sic_set_state(h, step: int, x, v_half):
    lib = load()
    px, kx, kx_ = _as_f64(x)
    pv, kv, kv_ = _as_f64(v_half)
    _check(lib.sic_set_state(h, int(step), px, pv, kx), "sic_set_state", h)


def sic_set_state_noalloc(h, step: int, x, v_half):
    lib = load()
    px, kx, kx_ = _as_f64(x)
    pv, kv, kv_ = _as_f64(v_half)
    _check(lib.sic_set_state_noalloc(h, int(step), px, pv, kx), "sic_set_state_noalloc", h)


def sic_refine(h, l_max: float) -> int:
    """One refinement pass; returns the number of tracers inserted."""
    n = ctypes.c_int64(0)
    _check(load().sic_refine(h, float(l_max), ctypes.byref(n)), "sic_refine", h)
    return n.value


def sic_get_layout(h, n_sheets: int):
    """(tracers per sheet, total)."""
    nt = np.zeros(int(n_sheets), dtype=np.int32)
    tot = ctypes.c_int64(0)
    _check(load().sic_get_layout(h, nt.ctypes.data_as(ctypes.c_void_p), ctypes.byref(tot)), "sic_get_layout", h)
    return nt, tot.value


def sic_get_charges(h, n_tracers_total: int, out=None):
    if out is None:
        out = np.zeros(int(n_tracers_total))
    pc, kc, _ = _as_f64(out)
    _check(load().sic_get_charges(h, pc, kc), "sic_get_charges", h)
    return out


def sic_load_state(h, step: int, n_tracers, x, v_half, seg_charges=None):
    lib = load()
    nt = np.ascontiguousarray(n_tracers, dtype=np.int32)
    px, kx, kx_ = _as_f64(x)
    pv, kv, kv_ = _as_f64(v_half)
    pc, kc, kc_ = _as_f64(seg_charges) if seg_charges is not None else (None, kx, None)
    if kx != kv or kx != kc:
        raise ValueError("x, v_half and seg_charges must live in the same memory")
    _check(lib.sic_load_state(h, int(step), nt.ctypes.data_as(ctypes.c_void_p), px, pv, pc, kx), "sic_load_state",
           h)


def sic_destroy(h):
    if h:
        load().sic_destroy(h)


def sic_last_error(h) -> str:
    return (load().sic_last_error(h) or b"").decode()


def sic_set_tuning(h, tile_chunks=0, block_threads=0, grid_blocks=0, fused_only=0):
    t = sic_tuning(int(tile_chunks), int(block_threads), int(grid_blocks), int(fused_only))
    _check(load().sic_set_tuning(h, ctypes.byref(t)), "sic_set_tuning", h)


def sic_get_tuning(h) -> dict:
    t = sic_tuning()
    _check(load().sic_get_tuning(h, ctypes.byref(t)), "sic_get_tuning", h)
    return dict(tile_chunks=t.tile_chunks, block_threads=t.block_threads, grid_blocks=t.grid_blocks,
                fused_only=t.fused_only)


def sic_set_timing(h, on: bool):
    _check(load().sic_set_timing(h, 1 if on else 0), "sic_set_timing", h)


def sic_last_step_path(h) -> int:
    p = ctypes.c_int32(0)
    _check(load().sic_last_step_path(h, ctypes.byref(p)), "sic_last_step_path", h)
    return p.value


def sic_last_timing(h):
    a, b = ctypes.c_double(0), ctypes.c_double(0)
    _check(load().sic_last_timing(h, ctypes.byref(a), ctypes.byref(b)), "sic_last_timing", h)
    return a.value, b.value


def sic_copy_bandwidth(n_bytes: int, iters: int = 5, stream=None) -> float:
    g = ctypes.c_double(0)
    _check(load().sic_copy_bandwidth(int(n_bytes), int(iters), _stream_ptr(stream), ctypes.byref(g)),
           "sic_copy_bandwidth")
    return g.value


# ------------------------------------------------------------------ batch

def sic_batch_create(budget_tracers, max_slots, max_cells, precision=SIC_FP64, history_rows=0, stream=None,
                     deposit_order=0, flags=0):
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    h = ctypes.c_void_p()
    rc = load().sic_batch_create(int(budget_tracers), int(max_slots), int(max_cells), int(precision),
                                 int(deposit_order), int(flags), int(history_rows), _stream_ptr(stream),
                                 ctypes.byref(h))
    _check(rc, "sic_batch_create")
    return h


def sic_batch_admit(b, L, n_cells, dt, n_tracers, q, closed, x0, v0, n_steps, precision=SIC_FP64,
                    raise_busy=True, deposit_order=0, seg_charges=None, l_max=0.0, max_tracers=0):
    """Returns the slot, or None when the batch is full (SIC_EBUSY) and raise_busy is False."""
    lib = load()
    cfg = make_config(L, n_cells, dt, precision, deposit_order=deposit_order, l_max=l_max,
                      max_tracers=max_tracers)
    sheets = make_sheets(n_tracers, q, closed)
    px, kx, kx_ = _as_f64(x0)
    pv, kv, kv_ = _as_f64(v0)
    pc, kc, kc_ = _as_f64(seg_charges) if seg_charges is not None else (None, kx, None)
    if kx != kv or kx != kc:
        raise ValueError("x0, v0 and seg_charges must live in the same memory")
    slot = ctypes.c_int32(-1)
    rc = lib.sic_batch_admit(b, ctypes.byref(cfg), sheets, len(sheets), px, pv, pc, kx, int(n_steps),
                             ctypes.byref(slot))
    if rc == 5 and not raise_busy:
        return None
    _check(rc, "sic_batch_admit", b, batch=True)
    return slot.value


def sic_batch_step(b, n_steps: int):
    _check(load().sic_batch_step(b, int(n_steps)), "sic_batch_step", b, batch=True)


def sic_batch_poll(b, cap: int = 65536):
    arr = (ctypes.c_int32 * cap)()
    n = ctypes.c_int32(0)
    _check(load().sic_batch_poll(b, arr, cap, ctypes.byref(n)), "sic_batch_poll", b, batch=True)
    return [arr[i] for i in range(n.value)]


def sic_batch_result(b, slot: int, n_cells: Optional[int] = None, history: bool = True):
    lib = load()
    last = sic_diag()
    rho = E = None
    prho = pE = None
    if n_cells:
        rho = np.zeros(int(n_cells))
        E = np.zeros(int(n_cells))
        prho = rho.ctypes.data_as(ctypes.c_void_p)
        pE = E.ctypes.data_as(ctypes.c_void_p)
    hist = None
    if history:
        n = ctypes.c_int64(0)
        _check(lib.sic_batch_result(b, int(slot), None, None, None, None, ctypes.byref(n)), "sic_batch_result", b,
               batch=True)
        hist = np.zeros(n.value, dtype=DIAG_DTYPE)
        _check(lib.sic_batch_result(b, int(slot), ctypes.byref(last), prho, pE, hist.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.byref(n)), "sic_batch_result", b, batch=True)
        hist = hist[: n.value]
    else:
        _check(lib.sic_batch_result(b, int(slot), ctypes.byref(last), prho, pE, None, None), "sic_batch_result",
               b, batch=True)
    return dict(last=_diag_dict(last), rho=rho, E=E, history=hist)


def sic_batch_get_state(b, slot: int, n_tracers_total: int, out_x=None, out_v=None):
    lib = load()
    if out_x is None:
        out_x = np.zeros(int(n_tracers_total))
        out_v = np.zeros(int(n_tracers_total))
    px, kx, _ = _as_f64(out_x)
    pv, kv, _ = _as_f64(out_v)
    step = ctypes.c_int64(0)
    _check(lib.sic_batch_get_state(b, int(slot), px, pv, ctypes.byref(step), kx), "sic_batch_get_state", b,
           batch=True)
    return out_x, out_v, step.value


def sic_batch_get_charges(b, slot: int, n_tracers_total: int, out=None):
    if out is None:
        out = np.zeros(int(n_tracers_total))
    pc, kc, _ = _as_f64(out)
    _check(load().sic_batch_get_charges(b, int(slot), pc, kc), "sic_batch_get_charges", b, batch=True)
    return out


def sic_batch_get_layout(b, slot: int, n_sheets: int):
    nt = np.zeros(int(n_sheets), dtype=np.int32)
    tot = ctypes.c_int64(0)
    _check(load().sic_batch_get_layout(b, int(slot), nt.ctypes.data_as(ctypes.c_void_p), ctypes.byref(tot)),
           "sic_batch_get_layout", b, batch=True)
    return nt, tot.value


def sic_batch_release(b, slot: int):
    _check(load().sic_batch_release(b, int(slot)), "sic_batch_release", b, batch=True)


def sic_batch_usage(b):
    t, s = ctypes.c_int64(0), ctypes.c_int32(0)
    _check(load().sic_batch_usage(b, ctypes.byref(t), ctypes.byref(s)), "sic_batch_usage", b, batch=True)
    return t.value, s.value


def sic_batch_set_tuning(b, tile_chunks=0, block_threads=0, grid_blocks=0):
    t = sic_tuning(int(tile_chunks), int(block_threads), int(grid_blocks), 0)
    _check(load().sic_batch_set_tuning(b, ctypes.byref(t)), "sic_batch_set_tuning", b, batch=True)


def sic_batch_get_tuning(b) -> dict:
    t = sic_tuning()
    _check(load().sic_batch_get_tuning(b, ctypes.byref(t)), "sic_batch_get_tuning", b, batch=True)
    return dict(tile_chunks=t.tile_chunks, block_threads=t.block_threads, grid_blocks=t.grid_blocks,
                fused_only=t.fused_only)


def sic_autotune(h, steps_per_trial: int = 3):
    t = sic_tuning()
    ms = ctypes.c_double(0)
    _check(load().sic_autotune(h, int(steps_per_trial), ctypes.byref(t), ctypes.byref(ms)), "sic_autotune", h)
    return dict(tile_chunks=t.tile_chunks, block_threads=t.block_threads, grid_blocks=t.grid_blocks,
                fused_only=t.fused_only), ms.value


def sic_batch_autotune(b, steps_per_trial: int = 3):
    t = sic_tuning()
    ms = ctypes.c_double(0)
    _check(load().sic_batch_autotune(b, int(steps_per_trial), ctypes.byref(t), ctypes.byref(ms)),
           "sic_batch_autotune", b, batch=True)
    return dict(tile_chunks=t.tile_chunks, block_threads=t.block_threads, grid_blocks=t.grid_blocks,
                fused_only=t.fused_only), ms.value


def sic_batch_set_timing(b, on: bool):
    _check(load().sic_batch_set_timing(b, 1 if on else 0), "sic_batch_set_timing", b, batch=True)


def sic_batch_last_timing(b):
    a, c = ctypes.c_double(0), ctypes.c_double(0)
    _check(load().sic_batch_last_timing(b, ctypes.byref(a), ctypes.byref(c)), "sic_batch_last_timing", b,
           batch=True)
    return a.value, c.value


def sic_batch_destroy(b):
    if b:
        load().sic_batch_destroy(b)


# ------------------------------------------------------------------ convenience

class Simulation:
    """Owns one sic_sim handle for an ``inputs.Problem``-like object."""

    def __init__(self, problem, precision=SIC_FP64, history_rows=0, stream=None, x0=None, v0=None,
                 deposit_order=0, seg_charges=None, l_max=0.0, max_tracers=0):
        self.problem = problem
        self.n = int(np.sum(problem.n_tracers, dtype=np.int64))
        if seg_charges is None:
            seg_charges = getattr(problem, "c_full", None)
        self.h = sic_init(problem.L, problem.n_cells, problem.dt, problem.n_tracers, problem.q, problem.closed,
                          problem.x0 if x0 is None else x0, problem.v0 if v0 is None else v0,
                          precision=precision, history_rows=history_rows, stream=stream,
                          deposit_order=deposit_order, seg_charges=seg_charges, l_max=l_max,
                          max_tracers=max_tracers)

    def step(self, n):
        try:
            sic_step(self.h, n)
        finally:
            # refinement may have grown the sheets, also when a later pass failed
            self._refresh_count()

    def _refresh_count(self):
        """Tracer total after refinement may have grown the sheets."""
        _, self.n = sic_get_layout(self.h, len(self.problem.n_tracers))

    def layout(self):
        return sic_get_layout(self.h, len(self.problem.n_tracers))

    def refine(self, l_max):
        added = sic_refine(self.h, l_max)
        self._refresh_count()
        return added

    def charges(self):
        return sic_get_charges(self.h, self.n)

    def load_state(self, step, n_tracers, x, v, seg_charges=None):
        sic_load_state(self.h, step, n_tracers, x, v, seg_charges)
        self.n = int(np.sum(n_tracers, dtype=np.int64))

    def deposit(self):
        sic_deposit(self.h)

    def solve(self):
        sic_solve_field(self.h)

    def push(self):
        sic_push(self.h)

    def diagnostics(self, history=True):
        return sic_diagnostics(self.h, self.problem.n_cells, history)

    def state(self):
        return sic_get_state(self.h, self.n)

    def set_state(self, step, x, v):
        sic_set_state(self.h, step, x, v)

    def close(self):
        if self.h:
            sic_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
