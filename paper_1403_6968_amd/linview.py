"""ctypes binding of liblinview (include/linview.h).

Argument marshalling only: every step of view creation, update and
re-evaluation runs in the library's HIP kernels.  PyTorch supplies device
memory (the caller-owned workspace and outputs) and the current stream.
The functions keep the C names; `View` is a small owner of a workspace and a
handle on top of them.

Loading fails loudly when the library has not been built: there is no
fallback path.
"""

from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LINVIEW_LIBRARY selects another build of the same library (the host
# AddressSanitizer build of the CPU tests); there is no fallback either way.
LIB_PATH = os.environ.get("LINVIEW_LIBRARY") or os.path.join(_HERE, "liblinview.so")

LV_OK, LV_EINVAL, LV_ENOMEM, LV_EDEVICE, LV_ESTATE = 0, 1, 2, 3, 4
LV_FP64, LV_FP32, LV_FP32_BF16SHADOW = 0, 1, 2
LV_WITH_SUMS = 1
LV_MODEL_EXP, LV_MODEL_LIN, LV_MODEL_SKIP = 0, 1, 2
LV_OLS_BETA, LV_OLS_INVERSE, LV_OLS_X = 0, 1, 2
LV_GENERAL_HYBRID, LV_GENERAL_FACTORED = 0, 1
LV_GLIN_REEVAL, LV_GLIN_HYBRID, LV_GLIN_INCR = 0, 1, 2
LV_STREAM_RMW, LV_STREAM_COPY, LV_STREAM_READ, LV_STREAM_WRITE = 0, 1, 2, 3

_MODE_DTYPE = {LV_FP64: torch.float64, LV_FP32: torch.float32, LV_FP32_BF16SHADOW: torch.float32}

EXPORTED = (
    "lv_status_str", "lv_last_error", "lv_view_footprint", "lv_view_create",
    "lv_view_update", "lv_view_update_batch", "lv_view_read", "lv_view_data",
    "lv_view_reanchor", "lv_view_stats", "lv_view_destroy", "lv_reeval_footprint",
    "lv_reeval", "lv_view_set_timing", "lv_view_set_pipeline", "lv_view_autotune", "lv_view_timing", "lv_view_write", "lv_view_drift_check",
    "lv_batch_footprint", "lv_batch_create", "lv_batch_inputs", "lv_batch_stage", "lv_batch_update",
    "lv_batch_destroy", "lv_server_create", "lv_server_view_bytes", "lv_server_set_hold", "lv_server_add_view",
    "lv_server_remove_view", "lv_server_view", "lv_server_now", "lv_server_submit", "lv_server_step",
    "lv_view_tile_rows", "lv_view_set_tile_rows", "lv_batch_tuning",
    "lv_view_footprint_ex", "lv_view_create_ex", "lv_view_read_sum",
    "lv_view_footprint_general", "lv_view_create_general", "lv_view_read_general",
    "lv_chain_footprint", "lv_chain_create", "lv_chain_update", "lv_chain_read", "lv_chain_powers",
    "lv_chain_destroy", "lv_ols_footprint", "lv_ols_create", "lv_ols_update", "lv_ols_update_row",
    "lv_ols_read", "lv_ols_info", "lv_ols_destroy",
    "lv_glin_footprint", "lv_glin_create", "lv_glin_update", "lv_glin_read", "lv_glin_destroy",
    "lv_server_poll", "lv_server_drain", "lv_server_stats", "lv_server_destroy",
    "lv_stream_probe", "lv_powers_update_noalloc", "lv_view_set_drift_check", "lv_server_set_admission_queue",
    "lv_tune_cache_save", "lv_tune_cache_load", "lv_tune_cache_clear",
)


class LinviewError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


class lv_stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("n_pad", ctypes.c_int64), ("ld", ctypes.c_int64),
        ("k", ctypes.c_int32), ("levels", ctypes.c_int32), ("r_max", ctypes.c_int32),
        ("mode", ctypes.c_int32), ("updates", ctypes.c_int64), ("reanchors", ctypes.c_int64),
        ("footprint", ctypes.c_size_t), ("drift_reanchors", ctypes.c_int64),
        ("last_residual", ctypes.c_double), ("drift_checks", ctypes.c_int64),
        ("drift_every", ctypes.c_int64), ("drift_tau", ctypes.c_double),
    ]


class lv_timing(ctypes.Structure):
    _fields_ = [
        ("fused_ms", ctypes.c_double), ("fused_launches", ctypes.c_int64),
        ("tail_ms", ctypes.c_double), ("tail_launches", ctypes.c_int64),
        ("top_ms", ctypes.c_double), ("top_launches", ctypes.c_int64),
    ]


class lv_server_counters(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
        ("coalesced_updates", ctypes.c_uint64), ("views", ctypes.c_int32),
        ("arena_free", ctypes.c_size_t), ("latency_p50_s", ctypes.c_double),
        ("latency_p99_s", ctypes.c_double), ("latency_max_s", ctypes.c_double),
        ("views_waiting", ctypes.c_int32), ("admitted_late", ctypes.c_uint64),
    ]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblinview.so (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    c = ctypes
    P, I64, I32, SZ = c.c_void_p, c.c_int64, c.c_int, c.c_size_t
    sig = {
        "lv_status_str": (c.c_char_p, [I32]),
        "lv_last_error": (c.c_char_p, []),
        "lv_view_footprint": (SZ, [I64, I32, I32, I32]),
        "lv_view_create": (I32, [P, I64, I64, I32, I32, I32, P, SZ, P, c.POINTER(P)]),
        "lv_view_update": (I32, [P, P, P, I64, I64, I64, P]),
        "lv_view_update_batch": (I32, [P, P, P, I64, I64, I64, I64, I64, I64, P]),
        "lv_view_read": (I32, [P, I32, P, I64, P]),
        "lv_view_data": (P, [P, I32, c.POINTER(I64)]),
        "lv_view_reanchor": (I32, [P, P]),
        "lv_view_stats": (I32, [P, c.POINTER(lv_stats)]),
        "lv_view_destroy": (None, [P]),
        "lv_reeval_footprint": (SZ, [I64, I32, I32]),
        "lv_reeval": (I32, [P, I64, I64, I32, P, P, I64, I64, I64, I32, P, I64, P, SZ, P]),
        "lv_view_set_timing": (I32, [P, I32]),
        "lv_view_set_pipeline": (I32, [P, I32]),
        "lv_view_autotune": (I32, [P, I32, I64, P, P]),
        "lv_view_write": (I32, [P, I32, P, I64, P]),
        "lv_view_drift_check": (I32, [P, P, c.c_double, P, P]),
        "lv_batch_footprint": (SZ, [c.POINTER(P), I32]),
        "lv_batch_create": (I32, [c.POINTER(P), I32, P, SZ, P, c.POINTER(P)]),
        "lv_batch_inputs": (I32, [P, I32, c.POINTER(P), c.POINTER(P), c.POINTER(I64)]),
        "lv_batch_stage": (I32, [P, I32, P, P, I64, I64, I64, P]),
        "lv_batch_update": (I32, [P, P]),
        "lv_batch_destroy": (None, [P]),
        "lv_server_create": (I32, [P, SZ, I32, I32, P, c.POINTER(P)]),
        "lv_server_view_bytes": (SZ, [P, I64, I32]),
        "lv_server_set_hold": (I32, [P, I32, c.c_double]),
        "lv_server_add_view": (I32, [P, P, I64, I64, I32, c.POINTER(I32)]),
        "lv_server_remove_view": (I32, [P, I32]),
        "lv_server_view": (P, [P, I32]),
        "lv_server_now": (c.c_double, [P]),
        "lv_server_submit": (I32, [P, I32, P, P, c.c_double, c.POINTER(c.c_uint64)]),
        "lv_server_step": (I32, [P, c.POINTER(I32)]),
        "lv_server_poll": (I32, [P, c.POINTER(c.c_uint64)]),
        "lv_server_drain": (I32, [P]),
        "lv_server_stats": (I32, [P, c.POINTER(lv_server_counters)]),
        "lv_server_destroy": (None, [P]),
        "lv_view_timing": (I32, [P, c.POINTER(lv_timing)]),
        "lv_view_tile_rows": (I32, [P, I32, c.POINTER(I32)]),
        "lv_view_set_tile_rows": (I32, [P, I32, I32]),
        "lv_batch_tuning": (I32, [P, c.POINTER(I32), c.POINTER(I32)]),
        "lv_view_footprint_ex": (SZ, [I64, I32, I32, I32, I32]),
        "lv_view_create_ex": (I32, [P, I64, I64, I32, I32, I32, I32, P, SZ, P, c.POINTER(P)]),
        "lv_view_read_sum": (I32, [P, I32, P, I64, P]),
        "lv_view_footprint_general": (SZ, [I64, I32, I32, I32, I64, I32, I32]),
        "lv_view_create_general": (I32, [P, I64, I64, I32, I32, I32, P, I64, P, I64, I64, I32, I32, P, SZ, P,
                                         c.POINTER(P)]),
        "lv_view_read_general": (I32, [P, I32, P, I64, P]),
        "lv_chain_footprint": (SZ, [I64, I32, I32, I32, I32, I32]),
        "lv_chain_create": (I32, [P, I64, I64, I32, I32, I32, I32, I32, P, SZ, P, c.POINTER(P)]),
        "lv_chain_update": (I32, [P, P, P, I64, I64, I64, P]),
        "lv_chain_read": (I32, [P, I32, P, I64, P]),
        "lv_chain_powers": (I32, [P, c.POINTER(I32), I32]),
        "lv_chain_destroy": (None, [P]),
        "lv_ols_footprint": (SZ, [I64, I64, I64, I32]),
        "lv_ols_create": (I32, [P, I64, I64, I64, P, I64, I64, I32, P, SZ, P, c.POINTER(P)]),
        "lv_ols_update": (I32, [P, P, P, P]),
        "lv_ols_update_row": (I32, [P, I64, P, P]),
        "lv_ols_read": (I32, [P, I32, P, I64, P]),
        "lv_ols_info": (I32, [P, c.POINTER(I32), c.POINTER(c.c_double), c.POINTER(c.c_double)]),
        "lv_ols_destroy": (None, [P]),
        "lv_glin_footprint": (SZ, [I64, I32, I32, I32, I64, I32]),
        "lv_glin_create": (I32, [P, I64, I64, I32, I32, I32, P, I64, P, I64, I64, I32, P, SZ, P, c.POINTER(P)]),
        "lv_glin_update": (I32, [P, P, P, I64, I64, I64, P]),
        "lv_glin_read": (I32, [P, I32, P, I64, P]),
        "lv_glin_destroy": (None, [P]),
        "lv_stream_probe": (I32, [I32, P, P, SZ, I32, I32, I32, P]),
        "lv_powers_update_noalloc": (I32, [c.POINTER(P), I64, I64, I32, I32, P, P, I64, I64, I64, P]),
        "lv_view_set_drift_check": (I32, [P, I64, c.c_double, P, P]),
        "lv_server_set_admission_queue": (I32, [P, I32]),
        "lv_tune_cache_save": (I32, [c.c_char_p]),
        "lv_tune_cache_load": (I32, [c.c_char_p, c.POINTER(I32)]),
        "lv_tune_cache_clear": (None, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int) -> None:
    if st != LV_OK:
        lib = load()
        raise LinviewError(st, f"{lib.lv_status_str(st).decode()}: {lib.lv_last_error().decode()}")


def _stream(stream, device) -> int:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _mat(x: torch.Tensor, dtype, name: str):
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {x.dtype}")
    if x.dim() != 2 or (x.stride(1) != 1 and x.shape[1] > 1):
        raise ValueError(f"{name} must be a row-major 2-D tensor")
    ld = x.stride(0) if x.shape[0] > 1 else x.shape[1]
    if ld < x.shape[1]:
        raise ValueError(f"{name} rows overlap")
    return x.data_ptr(), ld


# ---------------------------------------------------------------- C names

def lv_status_str(st: int) -> str:
    return load().lv_status_str(st).decode()


def lv_last_error() -> str:
    return load().lv_last_error().decode()


def lv_view_footprint(n: int, k: int, r_max: int, mode: int, flags: int = 0) -> int:
    return int(load().lv_view_footprint_ex(n, k, r_max, mode, flags))


def lv_view_create(A: torch.Tensor, k: int, r_max: int, mode: int, workspace: torch.Tensor,
                   stream=None, flags: int = 0) -> ctypes.c_void_p:
    lib = load()
    a, lda = _mat(A, _MODE_DTYPE[mode], "A")
    if A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    if workspace.device.type != "cuda" or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    h = ctypes.c_void_p()
    _check(lib.lv_view_create_ex(a, A.shape[0], lda, k, r_max, mode, flags, workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(),
                                 _stream(stream, A.device), ctypes.byref(h)))
    return h


def lv_view_footprint_general(n: int, k: int, r_max: int, mode: int, p: int,
                              strategy: int = LV_GENERAL_HYBRID, s: int = 0) -> int:
    return int(load().lv_view_footprint_general(n, k, r_max, mode, p, strategy, s))


def lv_view_create_general(A: torch.Tensor, k: int, r_max: int, mode: int, T0: torch.Tensor,
                           B: torch.Tensor, workspace: torch.Tensor, stream=None,
                           strategy: int = LV_GENERAL_HYBRID, s: int = 0) -> ctypes.c_void_p:
    lib = load()
    dtype = _MODE_DTYPE[mode]
    a, lda = _mat(A, dtype, "A")
    t, ldt = _mat(T0, dtype, "T0")
    b, ldb = _mat(B, dtype, "B")
    if A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    if T0.shape != B.shape or T0.shape[0] != A.shape[0]:
        raise ValueError("T0 and B must both be n x p")
    if workspace.device.type != "cuda" or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    h = ctypes.c_void_p()
    _check(lib.lv_view_create_general(a, A.shape[0], lda, k, r_max, mode, t, ldt, b, ldb, T0.shape[1], strategy,
                                      s, workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                      _stream(stream, A.device), ctypes.byref(h)))
    return h


def lv_view_read_general(view, index: int, out: torch.Tensor, dtype, stream=None) -> None:
    o, ldo = _mat(out, dtype, "out")
    _check(load().lv_view_read_general(view, index, o, ldo, _stream(stream, out.device)))


def lv_view_update(view, U: torch.Tensor, V: torch.Tensor, dtype, stream=None) -> None:
    u, ldu = _mat(U, dtype, "U")
    v, ldv = _mat(V, dtype, "V")
    if U.shape != V.shape:
        raise ValueError("U and V must have the same shape")
    _check(load().lv_view_update(view, u, v, U.shape[1], ldu, ldv, _stream(stream, U.device)))


def lv_view_update_batch(view, U: torch.Tensor, V: torch.Tensor, dtype, stream=None) -> None:
    """U, V: (count, n, r) device tensors, row-major per update."""
    if U.dim() != 3 or U.shape != V.shape:
        raise ValueError("U and V must be (count, n, r) tensors of one shape")
    if U.dtype != dtype or V.dtype != dtype:
        raise TypeError(f"U and V must be {dtype}")
    if U.shape[2] > 1 and (U.stride(2) != 1 or V.stride(2) != 1):
        raise ValueError("U and V must be row-major per update")
    if U.shape[1] > 1 and (U.stride(1) < U.shape[2] or V.stride(1) < V.shape[2]):
        raise ValueError("U and V rows overlap")
    ldu = U.stride(1) if U.shape[1] > 1 else U.shape[2]
    ldv = V.stride(1) if V.shape[1] > 1 else V.shape[2]
    _check(load().lv_view_update_batch(view, U.data_ptr(), V.data_ptr(), U.shape[2], U.shape[0],
                                       ldu, ldv, U.stride(0), V.stride(0),
                                       _stream(stream, U.device)))


def lv_view_read(view, power: int, out: torch.Tensor, dtype, stream=None) -> None:
    o, ldo = _mat(out, dtype, "out")
    _check(load().lv_view_read(view, power, o, ldo, _stream(stream, out.device)))


def lv_view_write(view, power: int, src: torch.Tensor, dtype, stream=None) -> None:
    a, lds = _mat(src, dtype, "src")
    _check(load().lv_view_write(view, power, a, lds, _stream(stream, src.device)))


def lv_view_drift_check(view, z: torch.Tensor, tau: float, residuals=None, stream=None) -> None:
    if z.dtype != torch.float64 or z.device.type != "cuda" or not z.is_contiguous():
        raise TypeError("z must be a contiguous float64 device vector")
    if residuals is not None and (residuals.dtype != torch.float64 or not residuals.is_contiguous()):
        raise TypeError("residuals must be a contiguous float64 device vector")
    _check(load().lv_view_drift_check(view, z.data_ptr(), float(tau),
                                      None if residuals is None else residuals.data_ptr(),
                                      _stream(stream, z.device)))


def lv_view_set_drift_check(view, every: int, tau: float = -1.0, z=None, stream=None, device=None) -> None:
    if z is not None and (z.dtype != torch.float64 or z.device.type != "cuda" or not z.is_contiguous()):
        raise TypeError("z must be a contiguous float64 device vector")
    dev = z.device if z is not None else (device or torch.device("cuda"))
    _check(load().lv_view_set_drift_check(view, int(every), float(tau), None if z is None else z.data_ptr(),
                                          _stream(stream, dev)))


def lv_view_data(view, power: int):
    ld = ctypes.c_int64()
    p = load().lv_view_data(view, power, ctypes.byref(ld))
    return p, ld.value


def lv_view_reanchor(view, stream=None, device=None) -> None:
    _check(load().lv_view_reanchor(view, _stream(stream, device)))


def lv_view_stats(view) -> dict:
    s = lv_stats()
    _check(load().lv_view_stats(view, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in lv_stats._fields_}


def lv_view_set_timing(view, enable: bool) -> None:
    _check(load().lv_view_set_timing(view, 1 if enable else 0))


def lv_view_set_pipeline(view, enable: bool) -> None:
    _check(load().lv_view_set_pipeline(view, 1 if enable else 0))


def lv_view_autotune(view, pipelined: bool = True, trial_updates: int = 24, stream=None, device=None) -> int:
    chosen = ctypes.c_int()
    _check(load().lv_view_autotune(view, 1 if pipelined else 0, int(trial_updates), _stream(stream, device),
                                   ctypes.byref(chosen)))
    return chosen.value


def lv_view_tile_rows(view, level: int) -> int:
    rows = ctypes.c_int()
    _check(load().lv_view_tile_rows(view, level, ctypes.byref(rows)))
    return rows.value


def lv_view_set_tile_rows(view, level: int, rows: int) -> None:
    _check(load().lv_view_set_tile_rows(view, level, rows))


def lv_tune_cache_save(path: str) -> None:
    _check(load().lv_tune_cache_save(os.fsencode(path)))


def lv_tune_cache_load(path: str) -> int:
    n = ctypes.c_int()
    _check(load().lv_tune_cache_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def lv_tune_cache_clear() -> None:
    load().lv_tune_cache_clear()


def lv_batch_tuning(batch) -> dict:
    t, h = ctypes.c_int(), ctypes.c_int()
    _check(load().lv_batch_tuning(batch, ctypes.byref(t), ctypes.byref(h)))
    return {"tuned_groups": t.value, "cache_hits": h.value}


def lv_view_timing(view) -> dict:
    t = lv_timing()
    _check(load().lv_view_timing(view, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in lv_timing._fields_}


def lv_view_destroy(view) -> None:
    load().lv_view_destroy(view)


def lv_stream_probe(kind: int, dst: torch.Tensor, src, nbytes: int, blocks: int, depth: int,
                    pipelined: bool = False, stream=None) -> None:
    """One launch of the streaming-ceiling kernel over nbytes of dst (and
    src); the caller times it with events on the stream."""
    if dst.device.type != "cuda" or (src is not None and src.device.type != "cuda"):
        raise TypeError("dst and src must be device tensors")
    if nbytes > dst.numel() * dst.element_size() and kind != LV_STREAM_READ:
        raise ValueError("dst is smaller than nbytes")
    if src is not None and nbytes > src.numel() * src.element_size():
        raise ValueError("src is smaller than nbytes")
    if kind == LV_STREAM_READ and dst.numel() * dst.element_size() < blocks * 1024:
        raise ValueError("READ needs blocks * 1024 bytes of dst")
    _check(load().lv_stream_probe(kind, dst.data_ptr(), None if src is None else src.data_ptr(), nbytes, blocks,
                                  depth, int(bool(pipelined)), _stream(stream, dst.device)))


def lv_powers_update_noalloc(powers, U: torch.Tensor, V: torch.Tensor, mode: int, stream=None) -> None:
    """One update of caller-held stored powers (A, A^2, ..., A^k, each n x n
    with one leading dimension) through the allocation-free entry point."""
    dtype = _MODE_DTYPE[mode]
    ptrs, lds = [], set()
    for i, P in enumerate(powers):
        p, ld = _mat(P, dtype, f"powers[{i}]")
        if P.shape[0] != P.shape[1] or P.shape[0] != powers[0].shape[0]:
            raise ValueError("every stored power must be n x n")
        ptrs.append(p)
        lds.add(ld)
    if len(lds) != 1:
        raise ValueError("the stored powers must share one leading dimension")
    u, ldu = _mat(U, dtype, "U")
    v, ldv = _mat(V, dtype, "V")
    arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
    _check(load().lv_powers_update_noalloc(arr, powers[0].shape[0], lds.pop(), 1 << (len(ptrs) - 1), mode, u, v,
                                           U.shape[1], ldu, ldv, _stream(stream, U.device)))


def lv_reeval_footprint(n: int, r_max: int, mode: int) -> int:
    return int(load().lv_reeval_footprint(n, r_max, mode))


def lv_reeval(A: torch.Tensor, k: int, U, V, mode: int, out: torch.Tensor,
              workspace: torch.Tensor, stream=None) -> None:
    dtype = _MODE_DTYPE[mode]
    a, lda = _mat(A, dtype, "A")
    o, ldo = _mat(out, dtype, "out")
    if U is None:
        u = v = None
        r = ldu = ldv = 0
    else:
        u, ldu = _mat(U, dtype, "U")
        v, ldv = _mat(V, dtype, "V")
        r = U.shape[1]
    _check(load().lv_reeval(a, A.shape[0], lda, k, u, v, r, ldu, ldv, mode, o, ldo,
                            workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                            _stream(stream, A.device)))


# ---------------------------------------------------------------- owner class

class View:
    """A view of A^k whose workspace is a torch device tensor."""

    def __init__(self, A: torch.Tensor, k: int, r_max: int = 1, mode: int | None = None,
                 stream=None, sums: bool = False, general=None, strategy: int = LV_GENERAL_HYBRID,
                 skip: int = 0):
        """general = (T0, B), both n x p: a view of the general form
        T_{i+1} = A T_i + B as well (implies sums), with hybrid or factored
        deltas (strategy).  skip = s > 0 (factored only): the powers and sums
        stop at s and T_2s, T_3s, ..., T_k follow the skip-s model."""
        if mode is None:
            mode = LV_FP64 if A.dtype == torch.float64 else LV_FP32
        self.mode = mode
        self.dtype = _MODE_DTYPE[mode]
        self.n = A.shape[0]
        self.k = k
        self.kp = skip if skip else k  # highest stored power
        self.device = A.device
        self.flags = LV_WITH_SUMS if sums or general is not None else 0
        self.p = 0
        if general is not None:
            T0, B = general
            self.p = T0.shape[1]
            nbytes = lv_view_footprint_general(self.n, k, r_max, mode, self.p, strategy, skip)
            if nbytes == 0:
                _check(load().lv_view_create_general(None, self.n, self.n, k, r_max, mode, None, self.p, None,
                                                     self.p, self.p, strategy, skip, None, 0, None,
                                                     ctypes.byref(ctypes.c_void_p())))
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
            self.handle = lv_view_create_general(A, k, r_max, mode, T0, B, self.workspace, stream, strategy, skip)
            return
        nbytes = lv_view_footprint(self.n, k, r_max, mode, self.flags)
        if nbytes == 0:
            # Reproduce the library's validation message.
            _check(load().lv_view_create_ex(None, self.n, self.n, k, r_max, mode, self.flags, None, 0, None,
                                            ctypes.byref(ctypes.c_void_p())))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
        self.handle = lv_view_create(A, k, r_max, mode, self.workspace, stream, self.flags)

    def update(self, U: torch.Tensor, V: torch.Tensor, stream=None) -> None:
        lv_view_update(self.handle, U, V, self.dtype, stream)

    def update_batch(self, U: torch.Tensor, V: torch.Tensor, stream=None) -> None:
        lv_view_update_batch(self.handle, U, V, self.dtype, stream)

    def read(self, power: int | None = None, stream=None) -> torch.Tensor:
        power = self.kp if power is None else power
        out = torch.empty(self.n, self.n, dtype=self.dtype, device=self.device)
        lv_view_read(self.handle, power, out, self.dtype, stream)
        return out

    def read_sum(self, index: int | None = None, stream=None) -> torch.Tensor:
        """Stored sum S_index = I + A + ... + A^(index - 1) (views with sums)."""
        index = self.kp if index is None else index
        out = torch.empty(self.n, self.n, dtype=self.dtype, device=self.device)
        _check(load().lv_view_read_sum(self.handle, index, out.data_ptr(), out.stride(0), _stream(stream, self.device)))
        return out

    def read_general(self, index: int | None = None, stream=None) -> torch.Tensor:
        """Stored T_index of the general form (general-form views)."""
        index = self.k if index is None else index
        out = torch.empty(self.n, max(self.p, 1), dtype=self.dtype, device=self.device)
        lv_view_read_general(self.handle, index, out, self.dtype, stream)
        return out

    def reanchor(self, stream=None) -> None:
        lv_view_reanchor(self.handle, stream, self.device)

    def write(self, power: int, src: torch.Tensor, stream=None) -> None:
        lv_view_write(self.handle, power, src, self.dtype, stream)

    def drift_check(self, z: torch.Tensor, tau: float, stream=None) -> torch.Tensor:
        """Residuals rho_j (device tensor, one per level below the top);
        re-anchors on the device when one exceeds tau."""
        m = len(self.powers()) - 1
        res = torch.zeros(max(m, 1), dtype=torch.float64, device=self.device)
        lv_view_drift_check(self.handle, z, tau, res if m > 0 else None, stream)
        return res[:m]

    def set_drift_check(self, every: int, tau: float = -1.0, z=None, stream=None) -> None:
        """Run the drift check after every `every`-th update (0: off);
        tau < 0 takes the mode's default bound."""
        lv_view_set_drift_check(self.handle, every, tau, z, stream, self.device)

    def stats(self) -> dict:
        return lv_view_stats(self.handle)

    def set_timing(self, enable: bool) -> None:
        lv_view_set_timing(self.handle, enable)

    def set_pipeline(self, enable: bool) -> None:
        """Pipelined (default) or sequential update_batch; equal results."""
        lv_view_set_pipeline(self.handle, enable)

    def autotune(self, pipelined: bool = True, trial_updates: int = 24, stream=None) -> int:
        """Tile rows chosen by timing zero updates (the view is unchanged)."""
        return lv_view_autotune(self.handle, pipelined, trial_updates, stream, self.device)

    def timing(self) -> dict:
        return lv_view_timing(self.handle)

    def tile_rows(self) -> list[int]:
        """Rows per tile of the level pass of each level below the top."""
        return [lv_view_tile_rows(self.handle, j) for j in range(len(self.powers()) - 1)]

    def set_tile_rows(self, rows) -> None:
        for j, r in enumerate(rows):
            lv_view_set_tile_rows(self.handle, j, r)

    def powers(self) -> list[int]:
        out, p = [], 1
        while p <= self.kp:
            out.append(p)
            p *= 2
        return out

    def general_indices(self) -> list[int]:
        """Indices i of the stored T_i (general-form views): 1, 2, 4, .., s,
        then 2s, 3s, .., k under the skip-s model."""
        return self.powers() + list(range(2 * self.kp, self.k + 1, self.kp))

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            torch.cuda.synchronize(self.device)
            lv_view_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _handles(views):
    arr = (ctypes.c_void_p * len(views))(*[v.handle.value for v in views])
    return arr


def lv_batch_footprint(views) -> int:
    return int(load().lv_batch_footprint(_handles(views), len(views)))


def lv_batch_create(views, workspace: torch.Tensor, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().lv_batch_create(_handles(views), len(views), workspace.data_ptr(),
                                  workspace.numel() * workspace.element_size(),
                                  _stream(stream, workspace.device), ctypes.byref(h)))
    return h


def lv_batch_stage(batch, i: int, U, V, dtype, stream=None, device=None) -> None:
    if U is None:
        _check(load().lv_batch_stage(batch, i, None, None, 0, 0, 0, _stream(stream, device)))
        return
    u, ldu = _mat(U, dtype, "U")
    v, ldv = _mat(V, dtype, "V")
    _check(load().lv_batch_stage(batch, i, u, v, U.shape[1], ldu, ldv, _stream(stream, U.device)))


def lv_batch_update(batch, stream=None, device=None) -> None:
    _check(load().lv_batch_update(batch, _stream(stream, device)))


def lv_batch_destroy(batch) -> None:
    load().lv_batch_destroy(batch)


class Batch:
    """One update per view per round for a list of `View`s of one mode; a
    round is one replay of a HIP graph captured at construction."""

    def __init__(self, views, stream=None):
        self.views = list(views)
        self.device = self.views[0].device
        self.dtype = self.views[0].dtype
        nbytes = lv_batch_footprint(self.views)
        if nbytes == 0:
            raise LinviewError(LV_EINVAL, lv_last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = lv_batch_create(self.views, self.workspace, stream)

    def stage(self, i: int, U=None, V=None, stream=None) -> None:
        lv_batch_stage(self.handle, i, U, V, self.dtype, stream, self.device)

    def update(self, stream=None) -> None:
        lv_batch_update(self.handle, stream, self.device)

    def tuning(self) -> dict:
        return lv_batch_tuning(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            torch.cuda.synchronize(self.device)
            lv_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop over views kept in one device arena (see linview.h):
    host-side rank-1 requests, per-view coalescing, continuous batching."""

    def __init__(self, arena_bytes: int, mode: int = LV_FP32, r_coalesce: int = 8,
                 device="cuda", stream=None):
        import numpy as _np
        self._np = _np
        self.mode = mode
        self.dtype = _MODE_DTYPE[mode]
        self.np_dtype = _np.float64 if mode == LV_FP64 else _np.float32
        self.device = torch.device(device)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        self._stream = _stream(stream, self.device)
        h = ctypes.c_void_p()
        _check(load().lv_server_create(self.arena.data_ptr(), arena_bytes, mode, r_coalesce,
                                       self._stream, ctypes.byref(h)))
        self.handle = h
        self.n = {}
        self.k = {}

    def view_bytes(self, n: int, k: int) -> int:
        return int(load().lv_server_view_bytes(self.handle, n, k))

    def set_hold(self, min_fill: int, max_wait_s: float) -> None:
        """Rounds take a view once it has min_fill requests queued or its
        oldest has waited max_wait_s (min_fill = 1: every pending view)."""
        _check(load().lv_server_set_hold(self.handle, min_fill, max_wait_s))

    def set_admission_queue(self, enable: bool) -> None:
        """Views that do not fit wait (A kept on the host) and are admitted
        when removals free room."""
        _check(load().lv_server_set_admission_queue(self.handle, int(bool(enable))))

    def add_view(self, A: torch.Tensor, k: int) -> int:
        a, lda = _mat(A, self.dtype, "A")
        vid = ctypes.c_int()
        _check(load().lv_server_add_view(self.handle, a, A.shape[0], lda, k, ctypes.byref(vid)))
        self.n[vid.value] = A.shape[0]
        self.k[vid.value] = k
        return vid.value

    def remove_view(self, vid: int) -> None:
        _check(load().lv_server_remove_view(self.handle, vid))
        self.n.pop(vid, None)
        self.k.pop(vid, None)

    def now(self) -> float:
        return float(load().lv_server_now(self.handle))

    def submit(self, vid: int, u, v, arrival: float = -1.0) -> int:
        u = self._np.ascontiguousarray(u, dtype=self.np_dtype)
        v = self._np.ascontiguousarray(v, dtype=self.np_dtype)
        if u.shape != (self.n[vid],) or v.shape != (self.n[vid],):
            raise ValueError("u and v must be vectors of the view's order")
        t = ctypes.c_uint64()
        _check(load().lv_server_submit(self.handle, vid, u.ctypes.data, v.ctypes.data, float(arrival),
                                       ctypes.byref(t)))
        return t.value

    def step(self) -> int:
        n = ctypes.c_int()
        _check(load().lv_server_step(self.handle, ctypes.byref(n)))
        return n.value

    def poll(self) -> int:
        c = ctypes.c_uint64()
        _check(load().lv_server_poll(self.handle, ctypes.byref(c)))
        return c.value

    def drain(self) -> None:
        _check(load().lv_server_drain(self.handle))

    def stats(self) -> dict:
        st = lv_server_counters()
        _check(load().lv_server_stats(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in lv_server_counters._fields_}

    def _view(self, vid: int) -> ctypes.c_void_p:
        h = load().lv_server_view(self.handle, vid)
        if not h:
            raise LinviewError(LV_EINVAL, f"no view {vid}")
        return ctypes.c_void_p(h)

    def view_handle(self, vid: int):
        """The admitted view's handle, or None (waiting or removed)."""
        h = load().lv_server_view(self.handle, vid)
        return ctypes.c_void_p(h) if h else None

    def set_drift_check(self, vid: int, every: int, tau: float = -1.0, z=None) -> None:
        """Periodic drift check of view vid every `every` of its (coalesced)
        updates; tau < 0 takes the mode's default bound."""
        lv_view_set_drift_check(self._view(vid), every, tau, z, self._stream, self.device)

    def view_stats(self, vid: int) -> dict:
        return lv_view_stats(self._view(vid))

    def read(self, vid: int, power: int) -> torch.Tensor:
        h = load().lv_server_view(self.handle, vid)
        if not h:
            raise LinviewError(LV_EINVAL, f"no view {vid}")
        n = self.n[vid]
        out = torch.empty(n, n, dtype=self.dtype, device=self.device)
        lv_view_read(ctypes.c_void_p(h), power, out, self.dtype, self._stream)
        return out

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            load().lv_server_destroy(self.handle)
            torch.cuda.synchronize(self.device)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reeval(A: torch.Tensor, k: int, U=None, V=None, stream=None) -> torch.Tensor:
    """(A + U V^T)^k by the library's re-evaluation path."""
    mode = LV_FP64 if A.dtype == torch.float64 else LV_FP32
    n = A.shape[0]
    r = 0 if U is None else U.shape[1]
    ws = torch.empty(lv_reeval_footprint(n, r, mode), dtype=torch.uint8, device=A.device)
    out = torch.empty(n, n, dtype=A.dtype, device=A.device)
    lv_reeval(A, k, U, V, mode, out, ws, stream)
    return out


class Chain:
    """A matrix-power view under the linear, skip-s or exponential model
    (LV_MODEL_*), for comparing IncrLin / IncrSkip-s with IncrExp."""

    def __init__(self, A: torch.Tensor, k: int, r_max: int = 1, model: int = LV_MODEL_LIN, s: int = 0,
                 mode: int | None = None, stream=None):
        if mode is None:
            mode = LV_FP64 if A.dtype == torch.float64 else LV_FP32
        self.mode, self.dtype = mode, _MODE_DTYPE[mode]
        self.n, self.k, self.device = A.shape[0], k, A.device
        lib = load()
        nbytes = int(lib.lv_chain_footprint(self.n, k, r_max, mode, model, s))
        if nbytes == 0:
            _check(lib.lv_chain_create(None, self.n, self.n, k, r_max, mode, model, s, None, 0, None,
                                       ctypes.byref(ctypes.c_void_p())))
        a, lda = _mat(A, self.dtype, "A")
        if A.shape[0] != A.shape[1]:
            raise ValueError("A must be square")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
        h = ctypes.c_void_p()
        _check(lib.lv_chain_create(a, self.n, lda, k, r_max, mode, model, s, self.workspace.data_ptr(), nbytes,
                                   _stream(stream, A.device), ctypes.byref(h)))
        self.handle = h

    def powers(self) -> list[int]:
        lib = load()
        cnt = lib.lv_chain_powers(self.handle, None, 0)
        buf = (ctypes.c_int * cnt)()
        lib.lv_chain_powers(self.handle, buf, cnt)
        return list(buf)

    def update(self, U: torch.Tensor, V: torch.Tensor, stream=None) -> None:
        u, ldu = _mat(U, self.dtype, "U")
        v, ldv = _mat(V, self.dtype, "V")
        if U.shape != V.shape:
            raise ValueError("U and V must have the same shape")
        _check(load().lv_chain_update(self.handle, u, v, U.shape[1], ldu, ldv, _stream(stream, self.device)))

    def read(self, power: int | None = None, stream=None) -> torch.Tensor:
        power = self.k if power is None else power
        out = torch.empty(self.n, self.n, dtype=self.dtype, device=self.device)
        _check(load().lv_chain_read(self.handle, power, out.data_ptr(), out.stride(0), _stream(stream, self.device)))
        return out

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            torch.cuda.synchronize(self.device)
            load().lv_chain_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ols:
    """Least squares beta = (X^T X)^{-1} X^T Y kept current under rank-1
    changes of X (Sherman-Morrison); X (m x n) and Y (m x p) device tensors."""

    def __init__(self, X: torch.Tensor, Y: torch.Tensor, mode: int | None = None, stream=None):
        if mode is None:
            mode = LV_FP64 if X.dtype == torch.float64 else LV_FP32
        self.mode, self.dtype = mode, _MODE_DTYPE[mode]
        self.m, self.n = X.shape
        self.p = Y.shape[1]
        self.device = X.device
        lib = load()
        nbytes = int(lib.lv_ols_footprint(self.m, self.n, self.p, mode))
        if nbytes == 0:
            _check(lib.lv_ols_create(None, self.m, self.n, self.n, None, self.p, self.p, mode, None, 0, None,
                                     ctypes.byref(ctypes.c_void_p())))
        x, ldx = _mat(X, self.dtype, "X")
        y, ldy = _mat(Y, self.dtype, "Y")
        if Y.shape[0] != self.m:
            raise ValueError("X and Y must have the same number of rows")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
        h = ctypes.c_void_p()
        _check(lib.lv_ols_create(x, self.m, self.n, ldx, y, self.p, ldy, mode, self.workspace.data_ptr(), nbytes,
                                 _stream(stream, X.device), ctypes.byref(h)))
        self.handle = h

    def _vec(self, x: torch.Tensor, length: int, name: str) -> int:
        if x.device.type != "cuda" or x.dtype != self.dtype or not x.is_contiguous() or x.numel() != length:
            raise ValueError(f"{name} must be a contiguous {self.dtype} device vector of {length} elements")
        return x.data_ptr()

    def update(self, u: torch.Tensor, v: torch.Tensor, stream=None) -> None:
        """Delta X = u v^T."""
        _check(load().lv_ols_update(self.handle, self._vec(u, self.m, "u"), self._vec(v, self.n, "v"),
                                    _stream(stream, self.device)))

    def update_row(self, row: int, dx: torch.Tensor, stream=None) -> None:
        """Delta X = e_row dx^T."""
        _check(load().lv_ols_update_row(self.handle, row, self._vec(dx, self.n, "dx"), _stream(stream, self.device)))

    def read(self, what: int = LV_OLS_BETA, stream=None) -> torch.Tensor:
        shape = {LV_OLS_BETA: (self.n, self.p), LV_OLS_INVERSE: (self.n, self.n), LV_OLS_X: (self.m, self.n)}[what]
        out = torch.empty(*shape, dtype=self.dtype, device=self.device)
        _check(load().lv_ols_read(self.handle, what, out.data_ptr(), shape[1], _stream(stream, self.device)))
        return out

    def info(self) -> dict:
        it, res, cond = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(load().lv_ols_info(self.handle, ctypes.byref(it), ctypes.byref(res), ctypes.byref(cond)))
        return {"iterations": it.value, "residual": res.value, "cond_inf": cond.value}

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            torch.cuda.synchronize(self.device)
            load().lv_ols_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GLin:
    """The general form T_{i+1} = A T_i + B under the linear model, every
    T_1 .. T_k stored, kept current by re-evaluation, hybrid or incremental
    evaluation (LV_GLIN_*)."""

    def __init__(self, A: torch.Tensor, k: int, T0: torch.Tensor, B: torch.Tensor, r_max: int = 1,
                 strategy: int = LV_GLIN_HYBRID, mode: int | None = None, stream=None):
        if mode is None:
            mode = LV_FP64 if A.dtype == torch.float64 else LV_FP32
        self.mode, self.dtype = mode, _MODE_DTYPE[mode]
        self.n, self.k, self.p, self.device = A.shape[0], k, T0.shape[1], A.device
        lib = load()
        nbytes = int(lib.lv_glin_footprint(self.n, k, r_max, mode, self.p, strategy))
        if nbytes == 0:
            _check(lib.lv_glin_create(None, self.n, self.n, k, r_max, mode, None, self.p, None, self.p, self.p,
                                      strategy, None, 0, None, ctypes.byref(ctypes.c_void_p())))
        a, lda = _mat(A, self.dtype, "A")
        t, ldt = _mat(T0, self.dtype, "T0")
        b, ldb = _mat(B, self.dtype, "B")
        if A.shape[0] != A.shape[1] or T0.shape != B.shape or T0.shape[0] != self.n:
            raise ValueError("A must be n x n and T0, B both n x p")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
        h = ctypes.c_void_p()
        _check(lib.lv_glin_create(a, self.n, lda, k, r_max, mode, t, ldt, b, ldb, self.p, strategy,
                                  self.workspace.data_ptr(), nbytes, _stream(stream, A.device), ctypes.byref(h)))
        self.handle = h

    def update(self, U: torch.Tensor, V: torch.Tensor, stream=None) -> None:
        u, ldu = _mat(U, self.dtype, "U")
        v, ldv = _mat(V, self.dtype, "V")
        if U.shape != V.shape:
            raise ValueError("U and V must have the same shape")
        _check(load().lv_glin_update(self.handle, u, v, U.shape[1], ldu, ldv, _stream(stream, self.device)))

    def read(self, i: int | None = None, stream=None) -> torch.Tensor:
        i = self.k if i is None else i
        out = torch.empty(self.n, self.p, dtype=self.dtype, device=self.device)
        _check(load().lv_glin_read(self.handle, i, out.data_ptr(), self.p, _stream(stream, self.device)))
        return out

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            torch.cuda.synchronize(self.device)
            load().lv_glin_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
