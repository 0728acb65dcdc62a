"""Thin Python binding of libmoa.so (include/moa.h), argument marshalling only.

Every function keeps the name of the C entry point it calls. Tensors are
PyTorch device tensors (torch is used for device memory and streams only);
every step of the computation runs in the library's HIP kernels. If the
library is missing this module raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmoa.so")

MOA_OK, MOA_ERR_INVALID, MOA_ERR_SHAPE, MOA_ERR_UNSUPPORTED = 0, 1, 2, 3
MOA_ERR_NOMEM, MOA_ERR_DEVICE, MOA_NOT_READY = 4, 5, 6
MOA_F64, MOA_F32 = 0, 1
MOA_PATH_AUTO, MOA_PATH_ONF, MOA_PATH_MFMA_F32 = 0, 1, 2
MOA_PATH_SPLIT_BF16, MOA_PATH_FP8_SCALED = 3, 4
MOA_FLAG_FP8_TWO_TERM = 0x1
MOA_FLAG_FP8_ONE_TERM = 0x2

PATHS = {"auto": MOA_PATH_AUTO, "onf": MOA_PATH_ONF, "mfma_f32": MOA_PATH_MFMA_F32,
         "split_bf16": MOA_PATH_SPLIT_BF16, "fp8": MOA_PATH_FP8_SCALED}


def MOA_FLAG_VARIANT(v: int) -> int:
    return (v + 1) << 8


def MOA_FLAG_SPLIT_K(c: int) -> int:
    return (c & 0xFF) << 16


MOA_FLAG_A_COL, MOA_FLAG_B_COL, MOA_FLAG_C_COL = 0x1000000, 0x2000000, 0x4000000


class MoaError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {status_name(status)}: {message}")
        self.status = status


class moa_gemm_desc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("p", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("path", ctypes.c_int32),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("accumulate", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class moa_plan_info(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("tile_m", ctypes.c_int32), ("tile_n", ctypes.c_int32),
                ("tile_k", ctypes.c_int32), ("wave_m", ctypes.c_int32),
                ("wave_n", ctypes.c_int32), ("lane_m", ctypes.c_int32),
                ("lane_n", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("workgroups", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("static_components", ctypes.c_int64),
                ("variant", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("split_k", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class moa_serve_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("slots", ctypes.c_int32),
                ("max_group", ctypes.c_int32), ("device", ctypes.c_int32),
                ("batch_window_us", ctypes.c_int32), ("pool_reserve_bytes", ctypes.c_int64)]


class moa_synth_request(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("p", ctypes.c_int64),
                ("path", ctypes.c_int32), ("flags", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class moa_serve_state(ctypes.Structure):
    _fields_ = [("held_bytes", ctypes.c_int64), ("peak_held_bytes", ctypes.c_int64),
                ("pool_bytes", ctypes.c_int64), ("peak_pool_bytes", ctypes.c_int64),
                ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("waiting", ctypes.c_int64)]


class moa_req_info(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("status", ctypes.c_int32), ("group_size", ctypes.c_int32)]


EXPORTS = [
    "moa_gemm", "moa_gemm_noalloc", "moa_gemm_grouped", "moa_gemm_grouped_variant", "moa_grouped_plan_query",
    "moa_autotune_grouped", "moa_plan_query", "moa_static_block_components",
    "moa_split_bf16", "moa_quantise_fp8", "moa_error_norm", "moa_serve_create",
    "moa_serve_submit", "moa_serve_submit_synthetic", "moa_serve_poll", "moa_serve_result", "moa_serve_read",
    "moa_serve_release", "moa_serve_drain", "moa_serve_stats", "moa_serve_destroy", "moa_fill_synthetic",
    "moa_status_string", "moa_last_error", "moa_trace_enable", "moa_trace_read",
    "moa_group_create", "moa_group_launch", "moa_group_destroy",
    "moa_autotune", "moa_autotune_save", "moa_autotune_load", "moa_autotune_clear",
    "moa_hadamard", "moa_kronecker", "moa_gemm_batched", "moa_diag_ring_loads",
]

MOA_KERNELS = {1: "onf_f64", 2: "onf_f32", 3: "mfma_f32", 4: "split_bf16", 5: "fp8", 6: "fp8_2term",
               7: "split_pack", 8: "fp8_quant", 9: "split_grouped", 10: "fp8_grouped", 11: "hadamard",
               12: "kronecker"}


class moa_trace_stat(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]

_lib = None


def lib():
    """Load libmoa.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2306_11148_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    P = ctypes.POINTER
    sig = {
        "moa_gemm": ([P(moa_gemm_desc), vp], i32),
        "moa_gemm_noalloc": ([P(moa_gemm_desc), vp], i32),
        "moa_gemm_grouped": ([P(moa_gemm_desc), i64, vp], i32),
        "moa_gemm_grouped_variant": ([P(moa_gemm_desc), i64, i32, vp], i32),
        "moa_grouped_plan_query": ([P(moa_gemm_desc), i64, P(i32), P(i32), P(i64)], i32),
        "moa_autotune_grouped": ([P(moa_gemm_desc), i64, i32, vp, P(i32), P(ctypes.c_double)], i32),
        "moa_plan_query": ([P(moa_gemm_desc), P(moa_plan_info)], i32),
        "moa_static_block_components": ([i64, i64, i64], i64),
        "moa_split_bf16": ([vp, i64, i64, vp, vp, vp], i32),
        "moa_quantise_fp8": ([vp, i64, i64, vp, i64, i32, vp, vp, vp, vp, vp, vp, vp], i32),
        "moa_error_norm": ([i64, i32, vp, vp, vp, vp], i32),
        "moa_serve_create": ([P(moa_serve_cfg), P(vp)], i32),
        "moa_serve_submit": ([vp, P(moa_gemm_desc), P(ctypes.c_uint64)], i32),
        "moa_serve_poll": ([vp, ctypes.c_uint64, P(moa_req_info)], i32),
        "moa_serve_submit_synthetic": ([vp, P(moa_synth_request), P(ctypes.c_uint64)], i32),
        "moa_serve_result": ([vp, ctypes.c_uint64, P(vp)], i32),
        "moa_serve_read": ([vp, ctypes.c_uint64, vp, i64], i32),
        "moa_serve_stats": ([vp, P(moa_serve_state)], i32),
        "moa_fill_synthetic": ([vp, i64, ctypes.c_uint64, ctypes.c_uint32, vp], i32),
        "moa_serve_release": ([vp, ctypes.c_uint64], i32),
        "moa_serve_drain": ([vp], i32),
        "moa_serve_destroy": ([vp], i32),
        "moa_status_string": ([i32], ctypes.c_char_p),
        "moa_last_error": ([], ctypes.c_char_p),
        "moa_trace_enable": ([i32], i32),
        "moa_autotune": ([P(moa_gemm_desc), i32, vp, P(moa_plan_info), P(ctypes.c_double)], i32),
        "moa_autotune_save": ([ctypes.c_char_p], i32),
        "moa_autotune_load": ([ctypes.c_char_p], i32),
        "moa_autotune_clear": ([], i32),
        "moa_group_create": ([P(moa_gemm_desc), i64, P(vp)], i32),
        "moa_group_launch": ([vp, vp], i32),
        "moa_group_destroy": ([vp], i32),
        "moa_trace_read": ([P(moa_trace_stat), i32, P(i32), i32], i32),
        "moa_hadamard": ([i64, i64, i32, vp, vp, vp, i32, vp], i32),
        "moa_kronecker": ([i64, i64, i64, i64, i32, vp, vp, vp, i32, vp], i32),
        "moa_gemm_batched": ([P(moa_gemm_desc), i64, i64, i64, i64, vp], i32),
        "moa_diag_ring_loads": ([P(moa_gemm_desc), P(i64), P(i64)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def status_name(s: int) -> str:
    return lib().moa_status_string(s).decode()


def moa_last_error() -> str:
    return lib().moa_last_error().decode()


def _check(status: int, where: str):
    if status != MOA_OK:
        raise MoaError(status, where, moa_last_error())


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return MOA_F64
    if t.dtype == torch.float32:
        return MOA_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _layout_flag(name, t, col_flag):
    """0 for a row-major (contiguous) 2-D tensor, col_flag for a column-major
    one (the transpose of a contiguous tensor, e.g. X.t()); anything else is
    refused."""
    if t.dim() != 2:
        raise ValueError(f"{name} must be a 2-D tensor")
    if t.is_contiguous():
        return 0
    if t.t().is_contiguous():
        return col_flag
    raise ValueError(f"{name} must be row-major (contiguous) or column-major (the transpose of a contiguous "
                     f"tensor), Eq. 4 and the gamma_col layout")


def make_desc(A, B, C, path=MOA_PATH_AUTO, accumulate=False, flags=0) -> moa_gemm_desc:
    """Descriptor for C (:= or +=) A.B from 2-D device tensors, each row-major
    (contiguous) or column-major (the transpose of a contiguous tensor); the
    layout flags follow from the strides."""
    flags |= (_layout_flag("A", A, MOA_FLAG_A_COL) | _layout_flag("B", B, MOA_FLAG_B_COL) |
              _layout_flag("C", C, MOA_FLAG_C_COL))
    m, n = A.shape
    if B.shape[0] != n or tuple(C.shape) != (m, B.shape[1]):
        raise ValueError(f"shapes {tuple(A.shape)} x {tuple(B.shape)} -> {tuple(C.shape)} do not conform")
    if isinstance(path, str):
        path = PATHS[path]
    dt = _dtype_code(A)
    if _dtype_code(B) != dt or _dtype_code(C) != dt:
        raise TypeError("A, B and C must share one dtype")
    return moa_gemm_desc(m, n, B.shape[1], dt, path, A.data_ptr() if A.numel() else None,
                         B.data_ptr() if B.numel() else None, C.data_ptr() if C.numel() else None,
                         int(bool(accumulate)), flags)


def moa_gemm(A, B, C, path=MOA_PATH_AUTO, accumulate=False, flags=0, stream=None):
    d = make_desc(A, B, C, path, accumulate, flags)
    _check(lib().moa_gemm(ctypes.byref(d), _stream_handle(stream)), "moa_gemm")
    return C


def moa_gemm_noalloc(A, B, C, path=MOA_PATH_AUTO, accumulate=False, flags=0, stream=None):
    d = make_desc(A, B, C, path, accumulate, flags)
    _check(lib().moa_gemm_noalloc(ctypes.byref(d), _stream_handle(stream)), "moa_gemm_noalloc")
    return C


MOA_NOALLOC_SCRATCH_BYTES = 64 << 20


def moa_gemm_desc_call(desc: moa_gemm_desc, stream=None) -> int:
    """Raw call with a prepared descriptor; returns the status code."""
    return lib().moa_gemm(ctypes.byref(desc), _stream_handle(stream))


def moa_gemm_grouped(descs, stream=None):
    arr = (moa_gemm_desc * len(descs))(*descs)
    _check(lib().moa_gemm_grouped(arr, len(descs), _stream_handle(stream)), "moa_gemm_grouped")


MOA_GROUPED_VARIANTS = 5


def moa_gemm_grouped_variant(descs, variant: int, stream=None):
    """moa_gemm_grouped with the persistent split-BF16 kernel forced (-1: planner choice)."""
    arr = (moa_gemm_desc * len(descs))(*descs)
    _check(lib().moa_gemm_grouped_variant(arr, len(descs), variant, _stream_handle(stream)),
           "moa_gemm_grouped_variant")


def moa_grouped_plan_query(descs) -> dict:
    arr = (moa_gemm_desc * len(descs))(*descs)
    v, t, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().moa_grouped_plan_query(arr, len(descs), ctypes.byref(v), ctypes.byref(t), ctypes.byref(n)),
           "moa_grouped_plan_query")
    return {"variant": v.value, "tuned": t.value, "persistent_members": n.value}


def moa_autotune_grouped(descs, reps: int = 3, stream=None):
    """Times every persistent split-BF16 kernel on this member list; returns (variant, best_ms)."""
    arr = (moa_gemm_desc * len(descs))(*descs)
    v, ms = ctypes.c_int32(), ctypes.c_double()
    _check(lib().moa_autotune_grouped(arr, len(descs), reps, _stream_handle(stream), ctypes.byref(v),
                                      ctypes.byref(ms)), "moa_autotune_grouped")
    return v.value, ms.value


def moa_plan_query(desc: moa_gemm_desc) -> dict:
    info = moa_plan_info()
    _check(lib().moa_plan_query(ctypes.byref(desc), ctypes.byref(info)), "moa_plan_query")
    return {f: getattr(info, f) for f, _ in moa_plan_info._fields_}


def moa_diag_ring_loads(desc: moa_gemm_desc) -> tuple[int, int]:
    """(loads checked per slab, violations) of the record-ring launch of desc's plan."""
    loads, bad = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().moa_diag_ring_loads(ctypes.byref(desc), ctypes.byref(loads), ctypes.byref(bad)),
           "moa_diag_ring_loads")
    return loads.value, bad.value


def moa_static_block_components(budget_bytes: int, elem_bytes: int, nblocks: int = 3) -> int:
    return lib().moa_static_block_components(budget_bytes, elem_bytes, nblocks)


def moa_split_bf16(X, hi, lo, stream=None):
    rows, cols = (X.shape if X.dim() == 2 else (1, X.numel()))
    _check(lib().moa_split_bf16(X.data_ptr(), rows, cols, hi.data_ptr(), lo.data_ptr(),
                                _stream_handle(stream)), "moa_split_bf16")


def moa_quantise_fp8(A, B, e, qA, f, qB, lA=None, lB=None, two_term=False, stream=None):
    m, n = A.shape
    p = B.shape[1]
    ptr = lambda t: t.data_ptr() if t is not None and t.numel() else None
    _check(lib().moa_quantise_fp8(ptr(A), m, n, ptr(B), p, int(bool(two_term)), ptr(e), ptr(qA),
                                  ptr(lA), ptr(f), ptr(qB), ptr(lB), _stream_handle(stream)),
           "moa_quantise_fp8")


def moa_error_norm(X, R, out, stream=None):
    _check(lib().moa_error_norm(X.numel(), _dtype_code(X), X.data_ptr(), R.data_ptr(),
                                out.data_ptr(), _stream_handle(stream)), "moa_error_norm")
    return out


# ------------------------------------------------------------------ serving --

def moa_serve_create(hbm_budget_bytes: int, slots: int = 4, max_group: int = 16, device: int = 0,
                     batch_window_us: int = 0, pool_reserve_bytes: int = 0):
    """Start a server; returns an opaque handle (int)."""
    cfg = moa_serve_cfg(hbm_budget_bytes, slots, max_group, device, batch_window_us, pool_reserve_bytes)
    h = ctypes.c_void_p()
    _check(lib().moa_serve_create(ctypes.byref(cfg), ctypes.byref(h)), "moa_serve_create")
    return h.value


def moa_serve_submit(srv, desc: moa_gemm_desc) -> int:
    t = ctypes.c_uint64()
    _check(lib().moa_serve_submit(srv, ctypes.byref(desc), ctypes.byref(t)), "moa_serve_submit")
    return t.value


def moa_serve_submit_synthetic(srv, m: int, n: int, p: int, path, seed: int, flags: int = 0) -> int:
    if isinstance(path, str):
        path = PATHS[path]
    req = moa_synth_request(m, n, p, path, flags, seed)
    t = ctypes.c_uint64()
    _check(lib().moa_serve_submit_synthetic(srv, ctypes.byref(req), ctypes.byref(t)),
           "moa_serve_submit_synthetic")
    return t.value


def moa_serve_result(srv, ticket: int) -> int:
    """Device address of a done request's C."""
    c = ctypes.c_void_p()
    _check(lib().moa_serve_result(srv, ticket, ctypes.byref(c)), "moa_serve_result")
    return c.value or 0


def moa_serve_read(srv, ticket: int, out):
    """Copies a done request's C into `out` (a C-contiguous numpy array or
    device tensor of m x p elements)."""
    if hasattr(out, "data_ptr"):
        ptr, nbytes = out.data_ptr(), out.numel() * out.element_size()
    else:
        ptr, nbytes = out.ctypes.data, out.nbytes
    _check(lib().moa_serve_read(srv, ticket, ptr, nbytes), "moa_serve_read")
    return out


def moa_serve_stats(srv) -> dict:
    st = moa_serve_state()
    _check(lib().moa_serve_stats(srv, ctypes.byref(st)), "moa_serve_stats")
    return {f: getattr(st, f) for f, _ in moa_serve_state._fields_}


def moa_fill_synthetic(X, seed: int, operand: int, stream=None):
    """Draws X (an FP32 device tensor) as operand `operand` of a request with `seed`."""
    _check(lib().moa_fill_synthetic(X.data_ptr() if X.numel() else None, X.numel(), seed, operand,
                                    _stream_handle(stream)), "moa_fill_synthetic")
    return X


def moa_serve_poll(srv, ticket: int):
    """Request info as a dict once done, None while it runs."""
    info = moa_req_info()
    s = lib().moa_serve_poll(srv, ticket, ctypes.byref(info))
    if s == MOA_NOT_READY:
        return None
    _check(s, "moa_serve_poll")
    return {f: getattr(info, f) for f, _ in moa_req_info._fields_}


def moa_serve_release(srv, ticket: int) -> bool:
    """Frees a completed ticket's record: True once released, False while the
    request still runs."""
    s = lib().moa_serve_release(srv, ticket)
    if s == MOA_NOT_READY:
        return False
    _check(s, "moa_serve_release")
    return True


def moa_serve_drain(srv):
    _check(lib().moa_serve_drain(srv), "moa_serve_drain")


def moa_serve_destroy(srv):
    _check(lib().moa_serve_destroy(srv), "moa_serve_destroy")


# ------------------------------------------------------------------ tracing --

def moa_trace_enable(on: bool = True):
    _check(lib().moa_trace_enable(int(bool(on))), "moa_trace_enable")


def moa_trace_read(reset: bool = False) -> dict:
    """{kernel name: (launches, total_ms)} for finished traced launches."""
    buf = (moa_trace_stat * 16)()
    n = ctypes.c_int32()
    _check(lib().moa_trace_read(buf, 16, ctypes.byref(n), int(bool(reset))), "moa_trace_read")
    return {MOA_KERNELS.get(buf[k].kernel, str(buf[k].kernel)): (buf[k].launches, buf[k].total_ms)
            for k in range(n.value)}


# ----------------------------------------------------------- prepared groups --

def moa_group_create(descs) -> int:
    arr = (moa_gemm_desc * len(descs))(*descs)
    h = ctypes.c_void_p()
    _check(lib().moa_group_create(arr, len(descs), ctypes.byref(h)), "moa_group_create")
    return h.value


def moa_group_launch(group, stream=None):
    _check(lib().moa_group_launch(group, _stream_handle(stream)), "moa_group_launch")


def moa_group_destroy(group):
    _check(lib().moa_group_destroy(group), "moa_group_destroy")


# ---------------------------------------------------------------- autotuner --

def moa_autotune(desc: moa_gemm_desc, reps: int = 3, stream=None):
    """Times every instantiation for desc's shape class; returns (plan, best_ms)."""
    info = moa_plan_info()
    ms = ctypes.c_double()
    _check(lib().moa_autotune(ctypes.byref(desc), reps, _stream_handle(stream), ctypes.byref(info),
                              ctypes.byref(ms)), "moa_autotune")
    return {f: getattr(info, f) for f, _ in moa_plan_info._fields_}, ms.value


def moa_autotune_save(path: str):
    _check(lib().moa_autotune_save(path.encode()), "moa_autotune_save")


def moa_autotune_load(path: str):
    _check(lib().moa_autotune_load(path.encode()), "moa_autotune_load")


def moa_autotune_clear():
    _check(lib().moa_autotune_clear(), "moa_autotune_clear")


# ----------------------------------------------------------- ipophp family --

def _rowmajor(name, t):
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")
    return t.data_ptr() if t.numel() else None


def moa_hadamard(A, B, C, accumulate=False, stream=None):
    """C := A * B elementwise (or C += A * B) for equal-shape 2-D tensors."""
    if A.dim() != 2 or tuple(A.shape) != tuple(B.shape) or tuple(A.shape) != tuple(C.shape):
        raise ValueError("A, B and C must be 2-D tensors of one shape")
    dt = _dtype_code(A)
    if _dtype_code(B) != dt or _dtype_code(C) != dt:
        raise TypeError("A, B and C must share one dtype")
    _check(lib().moa_hadamard(A.shape[0], A.shape[1], dt, _rowmajor("A", A), _rowmajor("B", B),
                              _rowmajor("C", C), int(bool(accumulate)), _stream_handle(stream)), "moa_hadamard")
    return C


def moa_kronecker(A, B, C, accumulate=False, stream=None):
    """C := A (x) B (or +=): A m x n, B p x q, C (m p) x (n q)."""
    m, n = A.shape
    p, q = B.shape
    if tuple(C.shape) != (m * p, n * q):
        raise ValueError(f"C must be {(m * p, n * q)}")
    dt = _dtype_code(A)
    if _dtype_code(B) != dt or _dtype_code(C) != dt:
        raise TypeError("A, B and C must share one dtype")
    _check(lib().moa_kronecker(m, n, p, q, dt, _rowmajor("A", A), _rowmajor("B", B), _rowmajor("C", C),
                               int(bool(accumulate)), _stream_handle(stream)), "moa_kronecker")
    return C


def moa_gemm_batched(A, B, C, path=MOA_PATH_AUTO, accumulate=False, flags=0, stream=None):
    """C[b] := A[b] B[b] for contiguous 3-D tensors (batch x m x n, batch x n x p,
    batch x m x p)."""
    if A.dim() != 3 or B.dim() != 3 or C.dim() != 3:
        raise ValueError("A, B and C must be 3-D tensors")
    batch = A.shape[0]
    if B.shape[0] != batch or C.shape[0] != batch:
        raise ValueError("batch sizes differ")
    d = make_desc(A[0], B[0], C[0], path, accumulate, flags) if batch else None
    if d is None:
        return C
    for name, t in (("A", A), ("B", B), ("C", C)):
        _rowmajor(name, t)
    _check(lib().moa_gemm_batched(ctypes.byref(d), batch, A.stride(0), B.stride(0), C.stride(0),
                                  _stream_handle(stream)), "moa_gemm_batched")
    return C
