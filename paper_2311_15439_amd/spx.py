"""ctypes binding of libspx.so: the same entry points as include/spx.h.

Argument marshalling only: every function checks that its tensors live on
the GPU with the expected dtype and layout, passes raw pointers and the
current HIP stream, and raises ``SpxError`` when the library returns a
non-OK status.  All arithmetic happens in the library's kernels; if the
library is missing, loading fails loudly (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass, field
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "spx.h")

SPX_OK, SPX_EINVAL, SPX_EALIGN, SPX_EUNSUPPORTED, SPX_EHIP = 0, 1, 2, 3, 4
SPX_F32, SPX_F16 = 0, 1
SPX_SIMPLEX, SPX_GRID = 0, 1
SPX_LAYOUT_HASHED, SPX_LAYOUT_SIZED = 0, 1
MAX_DIMS, MAX_LEVELS = 6, 32


class SpxError(RuntimeError):
    def __init__(self, status: int, fn: str, detail: str):
        super().__init__(f"{fn}: status {status} ({detail})")
        self.status = status


class spx_encoding(C.Structure):
    _fields_ = [("n_dims", C.c_int32), ("n_levels", C.c_int32), ("log2_T", C.c_int32),
                ("n_feat", C.c_int32), ("table_dtype", C.c_int32), ("cell", C.c_int32),
                ("equal_memory", C.c_int32), ("res", C.c_int32 * MAX_LEVELS), ("layout", C.c_int32)]


class spx_field(C.Structure):
    _fields_ = [("sigma", C.c_float * MAX_LEVELS), ("Fn", C.c_float), ("mask", C.c_uint32),
                ("n_dims", C.c_int32), ("n_levels", C.c_int32), ("cell", C.c_int32), ("d_out", C.c_int32),
                ("tables", C.c_void_p), ("W1", C.c_void_p), ("W2", C.c_void_p), ("W3", C.c_void_p)]


class spx_segment(C.Structure):
    _fields_ = [("pts", C.c_void_p), ("out", C.c_void_p), ("count", C.c_int64), ("first_tile", C.c_int64),
                ("field", C.c_int32), ("pad", C.c_int32)]


class spx_trace(C.Structure):
    _fields_ = [("events", C.c_void_p), ("names", C.c_void_p), ("bytes", C.c_void_p), ("capacity", C.c_int32),
                ("count", C.c_int32), ("only", C.c_char_p)]


class spx_mlp(C.Structure):
    _fields_ = [("d_in", C.c_int32), ("hidden", C.c_int32), ("d_out", C.c_int32)]


_P = C.c_void_p
_SIGNATURES = {
    "spx_abi_version": (C.c_int32, []),
    "spx_status_str": (C.c_char_p, [C.c_int]),
    "spx_last_error": (C.c_char_p, []),
    "spx_trace_set": (C.c_int, [_P]),
    "spx_level_resolutions": (C.c_int, [C.c_double, C.c_double, C.c_int32, _P]),
    "spx_level_scales": (C.c_int, [_P, _P]),
    "spx_hash_primes": (C.c_int, [_P]),
    "spx_table_layout": (C.c_int, [_P, _P, _P, _P, _P]),
    "spx_encode_fwd": (C.c_int, [_P, C.c_int64, _P, _P, _P, C.c_int32, _P]),
    "spx_encode_bwd": (C.c_int, [_P, C.c_int64, _P, _P, C.c_int32, _P, _P, C.c_size_t, _P]),
    "spx_encode_bwd_workspace": (C.c_int, [_P, C.c_int64, _P]),
    "spx_encode_bwd_adam": (C.c_int, [_P, C.c_int64, _P, _P, C.c_int32, _P, _P, _P, _P, C.c_float, C.c_float,
                                      C.c_float, C.c_float, C.c_int64, _P, C.c_size_t, _P]),
    "spx_encode_bwd_prepare": (C.c_int, [_P, C.c_int64, _P, _P, C.c_size_t, _P]),
    "spx_encode_bwd_prepared": (C.c_int, [_P, C.c_int64, _P, _P, C.c_int32, _P, _P, C.c_size_t, _P]),
    "spx_encode_bwd_adam_prepared": (C.c_int, [_P, C.c_int64, _P, _P, C.c_int32, _P, _P, _P, _P, C.c_float,
                                               C.c_float, C.c_float, C.c_float, C.c_int64, _P, C.c_size_t, _P]),
    "spx_encode_debug": (C.c_int, [_P, C.c_int64, _P, _P, _P, _P]),
    "spx_encode_gather_twin": (C.c_int, [_P, C.c_int64, _P, _P, _P, _P]),
    "spx_gather_probe": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int32, C.c_uint32, _P, _P]),
    "spx_encode_input_grad": (C.c_int, [_P, C.c_int64, _P, _P, _P, C.c_int32, _P, _P]),
    "spx_encode_mlp_fwd": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "spx_composite_fwd": (C.c_int, [C.c_int64, C.c_int32, _P, _P, _P, _P]),
    "spx_composite_bwd": (C.c_int, [C.c_int64, C.c_int32, _P, _P, _P, _P, _P]),
    "spx_cast_f32_f16": (C.c_int, [C.c_int64, _P, _P, _P]),
    "spx_adam_step": (C.c_int, [C.c_int64, _P, _P, _P, _P, _P, C.c_float, C.c_float, C.c_float,
                                C.c_float, C.c_int64, C.c_int32, _P]),
    "spx_field_init": (C.c_int, [_P, _P, _P, _P, _P, C.c_int32, _P]),
    "spx_field_query_batched": (C.c_int, [_P, C.c_int32, _P, C.c_int32, C.c_int64, _P]),
    "spx_mse_grad": (C.c_int, [C.c_int64, _P, _P, _P, C.c_float, _P]),
    "spx_mlp_fwd": (C.c_int, [_P, C.c_int64, _P, _P, _P, _P, _P, _P]),
    "spx_mlp_bwd_workspace": (C.c_int, [_P, C.c_int64, _P]),
    "spx_mlp_bwd": (C.c_int, [_P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "spx_encode_mlp_bwd_adam": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                          C.c_float, C.c_float, C.c_float, C.c_float, C.c_int64, _P, C.c_size_t,
                                          _P]),
    "spx_encode_mlp_bwd_workspace": (C.c_int, [_P, _P, C.c_int64, _P]),
    "spx_mlp_bwd_noalloc": (C.c_int, [_P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
}

_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    """Load libspx.so (built by ``python -m paper_2311_15439_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_15439_amd.build`")
        try:  # load torch's HIP runtime first so the library and torch share one runtime
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> list:
    """Names of the functions declared in include/spx.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(spx_\w+)\s*\(", text, re.M)))


def _check(status: int, fn: str) -> None:
    if status != SPX_OK:
        raise SpxError(status, fn, lib().spx_last_error().decode())


@dataclass
class Encoding:
    """Python view of spx_encoding.  ``res`` lists the level resolutions."""
    n_dims: int
    res: Sequence[int]
    log2_T: int
    n_feat: int = 2
    table_dtype: int = SPX_F16
    cell: int = SPX_SIMPLEX
    equal_memory: bool = False
    layout: int = SPX_LAYOUT_HASHED
    _c: spx_encoding = field(default=None, init=False, repr=False)
    _shape: tuple = field(default=None, init=False, repr=False)

    def __post_init__(self):
        e = spx_encoding()
        e.n_dims, e.n_levels, e.log2_T = self.n_dims, len(self.res), self.log2_T
        e.n_feat, e.table_dtype, e.cell = self.n_feat, self.table_dtype, self.cell
        e.equal_memory = int(self.equal_memory)
        e.layout = int(self.layout)
        for i, r in enumerate(list(self.res)[:MAX_LEVELS]):
            e.res[i] = int(r)
        self._c = e
        self._shape = (self.n_levels, 1 << self.log2_T, self.n_feat)
        if self.layout != SPX_LAYOUT_HASHED:
            self._shape = (spx_table_layout(self)["total_rows"], self.n_feat)

    @property
    def n_levels(self) -> int:
        return len(self.res)

    @property
    def n_vertices(self) -> int:
        return (1 << self.n_dims) if self.cell == SPX_GRID else self.n_dims + 1

    @property
    def table_shape(self):
        """[L, T, F] for the hashed layout; [rows of all levels, F] otherwise."""
        return self._shape

    def ref(self):
        return C.byref(self._c)


# --------------------------------------------------------------- helpers

def _torch():
    import torch
    return torch


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return SPX_F32
    if t.dtype == torch.float16:
        return SPX_F16
    raise TypeError(f"unsupported dtype {t.dtype}")


# --------------------------------------------------------------- host helpers

def spx_abi_version() -> int:
    return int(lib().spx_abi_version())


def spx_status_str(status: int) -> str:
    return lib().spx_status_str(status).decode()


def spx_last_error() -> str:
    return lib().spx_last_error().decode()


def spx_level_resolutions(n_min: float, growth: float, L: int):
    out = (C.c_int32 * L)()
    _check(lib().spx_level_resolutions(float(n_min), float(growth), L, C.cast(out, C.c_void_p)),
           "spx_level_resolutions")
    return [int(v) for v in out]


def spx_level_scales(enc: Encoding):
    out = (C.c_float * enc.n_levels)()
    _check(lib().spx_level_scales(enc.ref(), C.cast(out, C.c_void_p)), "spx_level_scales")
    return [float(v) for v in out]


def spx_table_layout(enc: Encoding):
    """Per level: rows, box extent, dense flag; total rows and row offsets."""
    L = enc.n_levels
    rows, ext, dense, total = (C.c_int64 * L)(), (C.c_int32 * L)(), (C.c_int32 * L)(), C.c_int64(0)
    _check(lib().spx_table_layout(enc.ref(), C.cast(rows, C.c_void_p), C.cast(ext, C.c_void_p),
                                  C.cast(dense, C.c_void_p), C.byref(total)), "spx_table_layout")
    r = [int(v) for v in rows]
    offs = [0]
    for v in r:
        offs.append(offs[-1] + v)
    return {"rows": r, "box_extent": [int(v) for v in ext], "dense": [bool(v) for v in dense],
            "total_rows": int(total.value), "offsets": offs}


def spx_hash_primes():
    out = (C.c_uint32 * MAX_DIMS)()
    _check(lib().spx_hash_primes(C.cast(out, C.c_void_p)), "spx_hash_primes")
    return [int(v) for v in out]


# --------------------------------------------------------------- encoding

def spx_encode_fwd(enc: Encoding, pts, tables, out, stream=None) -> None:
    """pts [N, n] float32; tables [L, T, F]; out [N, L*F] float32/float16."""
    torch = _torch()
    N = pts.shape[0]
    if pts.shape != (N, enc.n_dims) or tuple(tables.shape) != enc.table_shape:
        raise ValueError("pts or tables shape does not match the encoding")
    if tuple(out.shape) != (N, enc.n_levels * enc.n_feat):
        raise ValueError("out shape must be [N, L*F]")
    tdt = torch.float16 if enc.table_dtype == SPX_F16 else torch.float32
    _check(lib().spx_encode_fwd(enc.ref(), N, _dev(pts, torch.float32, "pts"), _dev(tables, tdt, "tables"),
                                _dev(out, None, "out"), _dtype_code(out), _stream(stream)), "spx_encode_fwd")


def spx_encode_bwd_workspace(enc: Encoding, N: int) -> int:
    out = C.c_size_t(0)
    _check(lib().spx_encode_bwd_workspace(enc.ref(), N, C.byref(out)), "spx_encode_bwd_workspace")
    return int(out.value)


def spx_encode_bwd_prepare(enc: Encoding, pts, workspace, stream=None) -> None:
    """The adjoint's counting pass (points only) into ``workspace``, for a
    following spx_encode_bwd_prepared / spx_encode_bwd_adam_prepared call on
    the same points and workspace (the caller orders the two streams)."""
    torch = _torch()
    N = pts.shape[0]
    if pts.shape != (N, enc.n_dims):
        raise ValueError("pts shape does not match the encoding")
    _check(lib().spx_encode_bwd_prepare(enc.ref(), N, _dev(pts, torch.float32, "pts"),
                                        _dev(workspace, torch.uint8, "workspace"), workspace.numel(),
                                        _stream(stream)), "spx_encode_bwd_prepare")


def spx_encode_bwd_prepared(enc: Encoding, pts, d_out, d_tables, workspace, stream=None) -> None:
    """spx_encode_bwd (binned) after spx_encode_bwd_prepare."""
    spx_encode_bwd(enc, pts, d_out, d_tables, workspace, stream, _prepared=True)


def spx_encode_bwd(enc: Encoding, pts, d_out, d_tables, workspace=None, stream=None, _prepared=False) -> None:
    """Accumulates into d_tables [L, T, F] float32 (caller zeroes it).  With a
    uint8 GPU ``workspace`` of spx_encode_bwd_workspace() bytes the binned
    path runs; without one, the atomic path."""
    torch = _torch()
    N = pts.shape[0]
    if pts.shape != (N, enc.n_dims) or tuple(d_tables.shape) != enc.table_shape:
        raise ValueError("pts or d_tables shape does not match the encoding")
    if tuple(d_out.shape) != (N, enc.n_levels * enc.n_feat):
        raise ValueError("d_out shape must be [N, L*F]")
    ws = None if workspace is None else _dev(workspace, torch.uint8, "workspace")
    nbytes = 0 if workspace is None else workspace.numel()
    name = "spx_encode_bwd_prepared" if _prepared else "spx_encode_bwd"
    _check(getattr(lib(), name)(enc.ref(), N, _dev(pts, torch.float32, "pts"), _dev(d_out, None, "d_out"),
                                _dtype_code(d_out), _dev(d_tables, torch.float32, "d_tables"), ws, nbytes,
                                _stream(stream)), name)


def spx_encode_bwd_adam_prepared(enc: Encoding, pts, d_out, param, m, v, param_f16=None, *, lr, beta1=0.9,
                                 beta2=0.99, eps=1e-15, step, workspace, stream=None) -> None:
    """spx_encode_bwd_adam after spx_encode_bwd_prepare."""
    spx_encode_bwd_adam(enc, pts, d_out, param, m, v, param_f16, lr=lr, beta1=beta1, beta2=beta2, eps=eps,
                        step=step, workspace=workspace, stream=stream, _prepared=True)


def spx_encode_bwd_adam(enc: Encoding, pts, d_out, param, m, v, param_f16=None, *, lr, beta1=0.9, beta2=0.99,
                        eps=1e-15, step, workspace, stream=None, _prepared=False) -> None:
    """Adjoint + Adam on the tables in one pass (no gradient table)."""
    torch = _torch()
    N = pts.shape[0]
    for t in (param, m, v) + ((param_f16,) if param_f16 is not None else ()):
        if tuple(t.shape) != enc.table_shape:
            raise ValueError("table state shape does not match the encoding")
    if tuple(d_out.shape) != (N, enc.n_levels * enc.n_feat):
        raise ValueError("d_out shape must be [N, L*F]")
    f = torch.float32
    name = "spx_encode_bwd_adam_prepared" if _prepared else "spx_encode_bwd_adam"
    _check(getattr(lib(), name)(enc.ref(), N, _dev(pts, f, "pts"), _dev(d_out, None, "d_out"), _dtype_code(d_out),
                                _dev(param, f, "param"), _dev(m, f, "m"), _dev(v, f, "v"),
                                None if param_f16 is None else _dev(param_f16, torch.float16, "param_f16"),
                                float(lr), float(beta1), float(beta2), float(eps), int(step),
                                _dev(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream)),
           name)


def spx_encode_debug(enc: Encoding, pts, idx=None, w=None, stream=None) -> None:
    """idx [N, L, V] int32 (slots, reinterpret as uint32); w [N, L, V] float32."""
    torch = _torch()
    N = pts.shape[0]
    shape = (N, enc.n_levels, enc.n_vertices)
    if idx is not None and tuple(idx.shape) != shape:
        raise ValueError("idx shape must be [N, L, V]")
    if w is not None and tuple(w.shape) != shape:
        raise ValueError("w shape must be [N, L, V]")
    _check(lib().spx_encode_debug(enc.ref(), N, _dev(pts, torch.float32, "pts"),
                                  None if idx is None else _dev(idx, torch.int32, "idx"),
                                  None if w is None else _dev(w, torch.float32, "w"), _stream(stream)),
           "spx_encode_debug")


def spx_encode_input_grad(enc: Encoding, pts, tables, d_out, d_pts, stream=None) -> None:
    """d_pts [N, n] float32 = d_out [N, L*F] contracted with d out / d pts."""
    torch = _torch()
    N = pts.shape[0]
    if pts.shape != (N, enc.n_dims) or tuple(tables.shape) != enc.table_shape or tuple(d_pts.shape) != (N, enc.n_dims):
        raise ValueError("pts, tables or d_pts shape does not match the encoding")
    if tuple(d_out.shape) != (N, enc.n_levels * enc.n_feat):
        raise ValueError("d_out shape must be [N, L*F]")
    tdt = torch.float16 if enc.table_dtype == SPX_F16 else torch.float32
    _check(lib().spx_encode_input_grad(enc.ref(), N, _dev(pts, torch.float32, "pts"), _dev(tables, tdt, "tables"),
                                       _dev(d_out, None, "d_out"), _dtype_code(d_out),
                                       _dev(d_pts, torch.float32, "d_pts"), _stream(stream)),
           "spx_encode_input_grad")


def spx_encode_gather_twin(enc: Encoding, pts, tables, out, stream=None) -> None:
    """Measurement reference: the forward's gathers in fixed walk order,
    summed without weights.  tables [L, T, 2] float16, out [N, 2L] float16."""
    torch = _torch()
    N = pts.shape[0]
    if pts.shape != (N, enc.n_dims) or tuple(tables.shape) != enc.table_shape:
        raise ValueError("pts or tables shape does not match the encoding")
    if tuple(out.shape) != (N, enc.n_levels * enc.n_feat):
        raise ValueError("out shape must be [N, L*F]")
    _check(lib().spx_encode_gather_twin(enc.ref(), N, _dev(pts, torch.float32, "pts"),
                                        _dev(tables, torch.float16, "tables"), _dev(out, torch.float16, "out"),
                                        _stream(stream)), "spx_encode_gather_twin")


def spx_gather_probe(table, n_threads: int, per_thread: int, seed: int, out, stream=None) -> None:
    """Measurement reference: per_thread uniformly random 4-byte gathers from
    `table` (a GPU tensor whose size in words is a power of two) per
    thread, their integer sum written to out [n_threads] int32."""
    torch = _torch()
    nbytes = table.numel() * table.element_size()
    if nbytes % 4 or out.numel() != n_threads:
        raise ValueError("table must hold whole 4-byte words and out n_threads entries")
    _check(lib().spx_gather_probe(_dev(table, None, "table"), nbytes // 4, int(n_threads), int(per_thread),
                                  int(seed) & 0xFFFFFFFF, _dev(out, torch.int32, "out"), _stream(stream)),
           "spx_gather_probe")


def spx_composite_fwd(raw, delta, rgba, stream=None) -> None:
    """raw [R, S, 4] float32, delta [R, S] float32 -> rgba [R, 4] float32."""
    torch = _torch()
    if raw.dim() != 3 or raw.shape[2] != 4 or tuple(delta.shape) != tuple(raw.shape[:2]):
        raise ValueError("raw must be [R, S, 4] and delta [R, S]")
    if tuple(rgba.shape) != (raw.shape[0], 4):
        raise ValueError("rgba must be [R, 4]")
    f = torch.float32
    _check(lib().spx_composite_fwd(raw.shape[0], raw.shape[1], _dev(raw, f, "raw"), _dev(delta, f, "delta"),
                                   _dev(rgba, f, "rgba"), _stream(stream)), "spx_composite_fwd")


def spx_composite_bwd(raw, delta, d_rgba, d_raw, stream=None) -> None:
    """d_raw [R, S, 4] = adjoint of spx_composite_fwd applied to d_rgba [R, 4]."""
    torch = _torch()
    if raw.dim() != 3 or raw.shape[2] != 4 or tuple(delta.shape) != tuple(raw.shape[:2]):
        raise ValueError("raw must be [R, S, 4] and delta [R, S]")
    if tuple(d_rgba.shape) != (raw.shape[0], 4) or tuple(d_raw.shape) != tuple(raw.shape):
        raise ValueError("d_rgba must be [R, 4] and d_raw like raw")
    f = torch.float32
    _check(lib().spx_composite_bwd(raw.shape[0], raw.shape[1], _dev(raw, f, "raw"), _dev(delta, f, "delta"),
                                   _dev(d_rgba, f, "d_rgba"), _dev(d_raw, f, "d_raw"), _stream(stream)),
           "spx_composite_bwd")


# --------------------------------------------------------------- elementwise

def spx_cast_f32_f16(src, dst, stream=None) -> None:
    torch = _torch()
    if src.numel() != dst.numel():
        raise ValueError("size mismatch")
    _check(lib().spx_cast_f32_f16(src.numel(), _dev(src, torch.float32, "src"), _dev(dst, torch.float16, "dst"),
                                  _stream(stream)), "spx_cast_f32_f16")


def spx_adam_step(param, grad, m, v, param_f16=None, *, lr, beta1=0.9, beta2=0.99, eps=1e-15, step,
                  zero_grad=False, stream=None) -> None:
    torch = _torch()
    n = param.numel()
    for t in (grad, m, v) + ((param_f16,) if param_f16 is not None else ()):
        if t.numel() != n:
            raise ValueError("Adam state size mismatch")
    _check(lib().spx_adam_step(n, _dev(param, torch.float32, "param"), _dev(grad, torch.float32, "grad"),
                               _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v"),
                               None if param_f16 is None else _dev(param_f16, torch.float16, "param_f16"),
                               float(lr), float(beta1), float(beta2), float(eps), int(step), int(bool(zero_grad)),
                               _stream(stream)), "spx_adam_step")


def spx_mse_grad(y, target, d_y, scale, stream=None) -> None:
    torch = _torch()
    n = y.numel()
    if target.numel() != n or d_y.numel() != n:
        raise ValueError("size mismatch")
    f = torch.float32
    _check(lib().spx_mse_grad(n, _dev(y, f, "y"), _dev(target, f, "target"), _dev(d_y, f, "d_y"), float(scale),
                              _stream(stream)), "spx_mse_grad")


# --------------------------------------------------------------- MLP

def make_mlp(d_in: int = 32, hidden: int = 64, d_out: int = 3) -> spx_mlp:
    m = spx_mlp()
    m.d_in, m.hidden, m.d_out = d_in, hidden, d_out
    return m


def spx_mlp_fwd(mlp: spx_mlp, x, W1, W2, W3, y, stream=None) -> None:
    torch = _torch()
    N = x.shape[0]
    if tuple(x.shape) != (N, mlp.d_in) or tuple(y.shape) != (N, mlp.d_out):
        raise ValueError("x must be [N, d_in] and y [N, d_out]")
    if (tuple(W1.shape) != (mlp.hidden, mlp.d_in) or tuple(W2.shape) != (mlp.hidden, mlp.hidden)
            or tuple(W3.shape) != (mlp.d_out, mlp.hidden)):
        raise ValueError("weight shapes do not match the network")
    h = torch.float16
    _check(lib().spx_mlp_fwd(C.byref(mlp), N, _dev(x, h, "x"), _dev(W1, h, "W1"), _dev(W2, h, "W2"),
                             _dev(W3, h, "W3"), _dev(y, torch.float32, "y"), _stream(stream)), "spx_mlp_fwd")


def spx_mlp_bwd_workspace(mlp: spx_mlp, N: int) -> int:
    out = C.c_size_t(0)
    _check(lib().spx_mlp_bwd_workspace(C.byref(mlp), N, C.byref(out)), "spx_mlp_bwd_workspace")
    return int(out.value)


def spx_mlp_bwd(mlp: spx_mlp, x, W1, W2, W3, d_y, d_x, dW1, dW2, dW3, workspace, stream=None) -> None:
    torch = _torch()
    N = x.shape[0]
    if tuple(d_y.shape) != (N, mlp.d_out):
        raise ValueError("d_y must be [N, d_out]")
    if d_x is not None and tuple(d_x.shape) != (N, mlp.d_in):
        raise ValueError("d_x must be [N, d_in]")
    h, f = torch.float16, torch.float32
    _check(lib().spx_mlp_bwd(C.byref(mlp), N, _dev(x, h, "x"), _dev(W1, h, "W1"), _dev(W2, h, "W2"),
                             _dev(W3, h, "W3"), _dev(d_y, f, "d_y"), None if d_x is None else _dev(d_x, f, "d_x"),
                             _dev(dW1, f, "dW1"), _dev(dW2, f, "dW2"), _dev(dW3, f, "dW3"),
                             _dev(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream)),
           "spx_mlp_bwd")


def spx_encode_mlp_bwd_workspace(enc: Encoding, mlp: spx_mlp, N: int) -> int:
    out = C.c_size_t(0)
    _check(lib().spx_encode_mlp_bwd_workspace(enc.ref(), C.byref(mlp), N, C.byref(out)),
           "spx_encode_mlp_bwd_workspace")
    return int(out.value)


def spx_encode_mlp_bwd_adam(enc: Encoding, mlp: spx_mlp, pts, x, W1, W2, W3, d_y, dW1, dW2, dW3, param, m, v,
                            param_f16=None, *, lr, beta1=0.9, beta2=0.99, eps=1e-15, step, workspace,
                            stream=None) -> None:
    """Network backward + encoding adjoint + Adam on the tables, with the
    network's input gradient computed inside the adjoint's scatter."""
    torch = _torch()
    N = pts.shape[0]
    for t in (param, m, v) + ((param_f16,) if param_f16 is not None else ()):
        if tuple(t.shape) != enc.table_shape:
            raise ValueError("table state shape does not match the encoding")
    if tuple(x.shape) != (N, mlp.d_in) or tuple(d_y.shape) != (N, mlp.d_out):
        raise ValueError("x must be [N, d_in] and d_y [N, d_out]")
    h, f = torch.float16, torch.float32
    _check(lib().spx_encode_mlp_bwd_adam(enc.ref(), C.byref(mlp), N, _dev(pts, f, "pts"), _dev(x, h, "x"),
                                         _dev(W1, h, "W1"), _dev(W2, h, "W2"), _dev(W3, h, "W3"), _dev(d_y, f, "d_y"),
                                         _dev(dW1, f, "dW1"), _dev(dW2, f, "dW2"), _dev(dW3, f, "dW3"),
                                         _dev(param, f, "param"), _dev(m, f, "m"), _dev(v, f, "v"),
                                         None if param_f16 is None else _dev(param_f16, h, "param_f16"),
                                         float(lr), float(beta1), float(beta2), float(eps), int(step),
                                         _dev(workspace, torch.uint8, "workspace"), workspace.numel(),
                                         _stream(stream)),
           "spx_encode_mlp_bwd_adam")


def spx_mlp_bwd_noalloc(mlp: spx_mlp, x, W1, W2, W3, d_y, d_x, dW1, dW2, dW3, stream=None) -> None:
    """spx_mlp_bwd with the library's static scratch instead of a workspace
    (nothing is allocated; calls overlapping on one GPU race)."""
    torch = _torch()
    N = x.shape[0]
    if tuple(d_y.shape) != (N, mlp.d_out):
        raise ValueError("d_y must be [N, d_out]")
    if d_x is not None and tuple(d_x.shape) != (N, mlp.d_in):
        raise ValueError("d_x must be [N, d_in]")
    h, f = torch.float16, torch.float32
    _check(lib().spx_mlp_bwd_noalloc(C.byref(mlp), N, _dev(x, h, "x"), _dev(W1, h, "W1"), _dev(W2, h, "W2"),
                                     _dev(W3, h, "W3"), _dev(d_y, f, "d_y"),
                                     None if d_x is None else _dev(d_x, f, "d_x"), _dev(dW1, f, "dW1"),
                                     _dev(dW2, f, "dW2"), _dev(dW3, f, "dW3"), _stream(stream)),
           "spx_mlp_bwd_noalloc")


# --------------------------------------------------------------- serving

def spx_field_init(enc: Encoding, tables, W1, W2, W3, d_out: int) -> spx_field:
    """Host descriptor of a resident field (tables and weights stay on the GPU)."""
    torch = _torch()
    out = spx_field()
    h = torch.float16
    _check(lib().spx_field_init(enc.ref(), _dev(tables, h, "tables"), _dev(W1, h, "W1"), _dev(W2, h, "W2"),
                                _dev(W3, h, "W3"), int(d_out), C.byref(out)), "spx_field_init")
    return out


def spx_encode_mlp_fwd(enc: Encoding, mlp: "spx_mlp", pts, tables, W1, W2, W3, out, feats=None, stream=None) -> None:
    """Fused training forward: out [N, d_out] float32 (and feats [N, 32]
    float16 if given) from pts [N, n]."""
    torch = _torch()
    N = pts.shape[0]
    if pts.shape != (N, enc.n_dims) or tuple(tables.shape) != enc.table_shape:
        raise ValueError("pts or tables shape does not match the encoding")
    if tuple(out.shape) != (N, mlp.d_out) or (feats is not None and tuple(feats.shape) != (N, 32)):
        raise ValueError("out must be [N, d_out] and feats [N, 32]")
    h = torch.float16
    _check(lib().spx_encode_mlp_fwd(enc.ref(), C.byref(mlp), N, _dev(pts, torch.float32, "pts"),
                                    _dev(tables, h, "tables"), _dev(W1, h, "W1"), _dev(W2, h, "W2"),
                                    _dev(W3, h, "W3"), None if feats is None else _dev(feats, h, "feats"),
                                    _dev(out, torch.float32, "out"), _stream(stream)), "spx_encode_mlp_fwd")


def as_bytes(structs) -> bytes:
    return b"".join(bytes(s) for s in structs)


def spx_field_query_batched(fields_dev, nfields: int, segs_dev, nseg: int, total_tiles: int, stream=None) -> None:
    """fields_dev / segs_dev: uint8 GPU tensors holding spx_field / spx_segment arrays."""
    torch = _torch()
    _check(lib().spx_field_query_batched(_dev(fields_dev, torch.uint8, "fields"), int(nfields),
                                         _dev(segs_dev, torch.uint8, "segs"), int(nseg), int(total_tiles),
                                         _stream(stream)), "spx_field_query_batched")


# --------------------------------------------------------------- tracing

class Trace:
    """Per-kernel timing of everything the library launches on this thread
    inside ``with Trace(...)``: name, algorithmic bytes and duration (ms)
    from HIP events on each kernel's launch stream.  ``only`` restricts the
    events to the kernels of one name."""

    def __init__(self, capacity: int = 256, only: str = None):
        torch = _torch()
        self.capacity = capacity
        self.events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * capacity)]
        s = torch.cuda.current_stream()
        for e in self.events:  # create the underlying HIP events
            e.record(s)
        torch.cuda.synchronize()
        self._ev = (C.c_void_p * (2 * capacity))(*[e.cuda_event for e in self.events])
        self._names = (C.c_char_p * capacity)()
        self._bytes = (C.c_double * capacity)()
        self.t = spx_trace()
        self.t.events = C.cast(self._ev, C.c_void_p)
        self.t.names = C.cast(self._names, C.c_void_p)
        self.t.bytes = C.cast(self._bytes, C.c_void_p)
        self.t.capacity = capacity
        self._only = only.encode() if only else None
        self.t.only = self._only

    def __enter__(self):
        self.t.count = 0
        _check(lib().spx_trace_set(C.byref(self.t)), "spx_trace_set")
        return self

    def __exit__(self, *exc):
        lib().spx_trace_set(None)
        return False

    def results(self):
        """[(name, bytes, ms)] in launch order (synchronises)."""
        _torch().cuda.synchronize()
        return [(self._names[i].decode(), float(self._bytes[i]), self.events[2 * i].elapsed_time(self.events[2 * i + 1]))
                for i in range(self.t.count)]
