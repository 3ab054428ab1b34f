"""CPU oracle for the multiresolution simplex hash encoding (arXiv 2311.15439).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the benchmark's CPU-baseline leg may import this package.  It wraps
``spx_oracle.c`` (plain C, built with gcc) through ctypes and shares no code
with the HIP library.

Every function returns numpy arrays; see ``spx_oracle.c`` for the definitions
and the section of the paper each follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spx_oracle.c")
_LIB = os.environ.get("SPX_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

SIMPLEX, GRID = 0, 1
F32, F16 = 0, 1
HASHED, SIZED = 0, 1  # table layouts (see spx_oracle.c)
MAX_DIM, MAX_LEVELS = 6, 32


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, so binary32 steps are the
    plain IEEE operations in program order)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_timing(dst: str) -> str:
    """Compile the same source for timing on the host that runs it:
    ``-O3 -march=native`` (same operation order, no contraction), into
    ``dst``.  The parity build above stays as it is."""
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", dst, _SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return dst


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (for example
    the timing build) from now on."""
    global _LIB, _lib
    _LIB, _lib = path, None
    lib()


def library_path() -> str:
    return _LIB


class _Enc(C.Structure):
    _fields_ = [("n_dims", C.c_int), ("n_levels", C.c_int), ("log2_T", C.c_int),
                ("n_feat", C.c_int), ("table_dtype", C.c_int), ("cell", C.c_int),
                ("res", C.c_int32 * MAX_LEVELS), ("equal_memory", C.c_int), ("layout", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        for name, res, args in [
            ("orc_skew_factor", C.c_double, [C.c_int]),
            ("orc_unskew_factor", C.c_double, [C.c_int]),
            ("orc_adjust_scale", C.c_double, [C.c_int]),
            ("orc_equal_memory_factor", C.c_double, [C.c_int]),
            ("orc_level_resolutions", None, [C.c_double, C.c_double, C.c_int, P]),
            ("orc_level_scales", None, [C.c_int, C.c_int, P, C.c_int, C.c_int, P]),
            ("orc_hash_primes", None, [P]),
            ("orc_hash", C.c_uint32, [P, C.c_int, C.c_int]),
            ("orc_f16_to_f64", C.c_double, [C.c_uint16]),
            ("orc_f64_to_f16", C.c_uint16, [C.c_double]),
            ("orc_round_bf16", C.c_double, [C.c_double]),
            ("orc_encode_debug", None, [P, C.c_int64, P, P, P, P, P, P]),
            ("orc_table_layout", None, [P, P, P, P]),
            ("orc_vertex_slot", C.c_uint32, [P, C.c_int, P]),
            ("orc_encode_fwd", None, [P, C.c_int64, P, P, P]),
            ("orc_encode_fwd_absmag", None, [P, C.c_int64, P, P, P]),
            ("orc_encode_bwd", None, [P, C.c_int64, P, P, P, P, P]),
            ("orc_mlp_fwd", None, [C.c_int64, C.c_int, C.c_int, C.c_int, P, P, P, P, P, P]),
            ("orc_mlp_bwd", None, [C.c_int64, C.c_int, C.c_int, C.c_int, P, P, P, P, P, C.c_int, P, P, P,
                                   P, P, P, P, P, P]),
            ("orc_adam_step", None, [C.c_int64, P, P, P, P, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_int64, P]),
            ("orc_cast_f32_f16", None, [C.c_int64, P, P]),
            ("orc_mse_grad", None, [C.c_int64, P, P, C.c_double, P]),
            ("orc_encode_input_grad", None, [P, C.c_int64, P, P, P, P, P]),
            ("orc_composite_fwd", None, [C.c_int64, C.c_int, P, P, P]),
            ("orc_set_threads", None, [C.c_int]),
            ("orc_max_threads", C.c_int, []),
            ("orc_composite_bwd", None, [C.c_int64, C.c_int, P, P, P, P, P]),
        ]:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class Encoding:
    """Hyper-parameters of one encoding (mirrors the GPU descriptor by value
    only).  ``res`` holds the integer level resolutions N_l."""
    n_dims: int
    res: list
    log2_T: int
    n_feat: int = 2
    table_dtype: int = F32
    cell: int = SIMPLEX
    equal_memory: bool = False
    layout: int = HASHED

    @property
    def n_levels(self) -> int:
        return len(self.res)

    @property
    def n_vertices(self) -> int:
        return (1 << self.n_dims) if self.cell == GRID else self.n_dims + 1

    def _c(self) -> _Enc:
        e = _Enc()
        e.n_dims, e.n_levels, e.log2_T = self.n_dims, self.n_levels, self.log2_T
        e.n_feat, e.table_dtype, e.cell = self.n_feat, self.table_dtype, self.cell
        for i, r in enumerate(self.res):
            e.res[i] = int(r)
        e.equal_memory = int(self.equal_memory)
        e.layout = int(self.layout)
        return e

    @property
    def table_shape(self):
        """[L, T, F] for the hashed layout, [all rows, F] for the sized one."""
        if self.layout == HASHED:
            return (self.n_levels, 1 << self.log2_T, self.n_feat)
        return (int(table_layout(self)["offsets"][-1]), self.n_feat)


# --- constants ---------------------------------------------------------------

def skew_factor(n): return lib().orc_skew_factor(n)
def unskew_factor(n): return lib().orc_unskew_factor(n)
def adjust_scale(n): return lib().orc_adjust_scale(n)
def equal_memory_factor(n): return lib().orc_equal_memory_factor(n)


def level_resolutions(n_min: float, growth: float, L: int) -> np.ndarray:
    out = np.zeros(L, np.int32)
    lib().orc_level_resolutions(float(n_min), float(growth), L, _p(out))
    return out


def level_scales(n: int, res, cell: int = SIMPLEX, equal_memory: bool = False) -> np.ndarray:
    r = np.ascontiguousarray(res, np.int32)
    out = np.zeros(len(r), np.float32)
    lib().orc_level_scales(n, len(r), _p(r), cell, int(equal_memory), _p(out))
    return out


def hash_primes() -> np.ndarray:
    out = np.zeros(MAX_DIM, np.uint32)
    lib().orc_hash_primes(_p(out))
    return out


def hash_vertex(v, log2_T: int) -> int:
    a = np.ascontiguousarray(v, np.int32)
    return int(lib().orc_hash(_p(a), len(a), log2_T))


def f16_bits(x: float) -> int: return int(lib().orc_f64_to_f16(float(x)))
def f16_value(bits: int) -> float: return float(lib().orc_f16_to_f64(int(bits)))
def round_bf16(x: float) -> float: return float(lib().orc_round_bf16(float(x)))


# --- encoding ------------------------------------------------------------------

def _pts(pts, n):
    a = np.ascontiguousarray(pts, np.float32)
    assert a.ndim == 2 and a.shape[1] == n
    return a


def table_layout(e: Encoding):
    """Per level: rows, box extent per axis, dense flag; and the row offsets
    (offsets[l] is level l's first row, offsets[L] all rows)."""
    L = e.n_levels
    rows = np.zeros(L, np.int64)
    ext = np.zeros(L, np.int32)
    dense = np.zeros(L, np.int32)
    ce = e._c()
    lib().orc_table_layout(C.byref(ce), _p(rows), _p(ext), _p(dense))
    return dict(rows=rows, extent=ext, dense=dense.astype(bool), offsets=np.concatenate([[0], np.cumsum(rows)]))


def vertex_slot(e: Encoding, level: int, v) -> int:
    """Row of lattice vertex v within the level's table."""
    a = np.ascontiguousarray(v, np.int32)
    ce = e._c()
    return int(lib().orc_vertex_slot(C.byref(ce), int(level), _p(a)))


def _tables(e: Encoding, tables):
    dt = np.uint16 if e.table_dtype == F16 else np.float32
    t = np.ascontiguousarray(tables)
    if t.dtype == np.float16:
        t = t.view(np.uint16)
    assert t.dtype == dt, (t.dtype, dt)
    assert t.size == int(np.prod(e.table_shape))
    return t


def encode_debug(e: Encoding, pts):
    """Per point and level: vertex coordinates, hash slots, binary64 and
    binary32 weights, and the scaled point p."""
    x = _pts(pts, e.n_dims)
    N, L, V, n = len(x), e.n_levels, e.n_vertices, e.n_dims
    verts = np.zeros((N, L, V, n), np.int32)
    idx = np.zeros((N, L, V), np.uint32)
    w64 = np.zeros((N, L, V), np.float64)
    w32 = np.zeros((N, L, V), np.float32)
    p = np.zeros((N, L, n), np.float32)
    ce = e._c()
    lib().orc_encode_debug(C.byref(ce), N, _p(x), _p(verts), _p(idx), _p(w64), _p(w32), _p(p))
    return dict(verts=verts, idx=idx, w64=w64, w32=w32, p=p)


def encode_fwd(e: Encoding, pts, tables) -> np.ndarray:
    """Encoded features [N, L*F] in binary64."""
    x = _pts(pts, e.n_dims)
    t = _tables(e, tables)
    out = np.zeros((len(x), e.n_levels * e.n_feat), np.float64)
    ce = e._c()
    lib().orc_encode_fwd(C.byref(ce), len(x), _p(x), _p(t), _p(out))
    return out


def encode_fwd_absmag(e: Encoding, pts, tables) -> np.ndarray:
    """sum_k |w_k t_k| per output (the scale the forward error is stated against)."""
    x = _pts(pts, e.n_dims)
    t = _tables(e, tables)
    out = np.zeros((len(x), e.n_levels * e.n_feat), np.float64)
    ce = e._c()
    lib().orc_encode_fwd_absmag(C.byref(ce), len(x), _p(x), _p(t), _p(out))
    return out


def encode_bwd(e: Encoding, pts, d_out, with_stats: bool = False):
    """Table gradient [L, T, F] in binary64 for output gradient d_out [N, L*F].
    With ``with_stats`` also returns sum |w d_out| and the contribution count
    per slot."""
    x = _pts(pts, e.n_dims)
    d = np.ascontiguousarray(d_out, np.float64)
    assert d.shape == (len(x), e.n_levels * e.n_feat)
    shape = e.table_shape
    g = np.zeros(shape, np.float64)
    absmag = np.zeros(shape, np.float64) if with_stats else None
    count = np.zeros(shape, np.int64) if with_stats else None
    ce = e._c()
    lib().orc_encode_bwd(C.byref(ce), len(x), _p(x), _p(d), _p(g), _p(absmag), _p(count))
    return (g, absmag, count) if with_stats else g


# --- MLP -----------------------------------------------------------------------

def _h(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.float16:
        a = a.view(np.uint16)
    assert a.dtype == np.uint16
    return a


def mlp_fwd(x, W1, W2, W3, with_absmag: bool = False):
    """x [N, d_in] binary16; W1 [H, d_in], W2 [H, H], W3 [d_out, H] binary16.
    Returns the output [N, d_out] in binary64 (and its magnitude with the
    ReLU pattern applied)."""
    x, W1, W2, W3 = _h(x), _h(W1), _h(W2), _h(W3)
    N, d_in = x.shape
    H, d_out = W1.shape[0], W3.shape[0]
    assert W1.shape == (H, d_in) and W2.shape == (H, H) and W3.shape == (d_out, H)
    out = np.zeros((N, d_out), np.float64)
    mag = np.zeros((N, d_out), np.float64) if with_absmag else None
    lib().orc_mlp_fwd(N, d_in, H, d_out, _p(x), _p(W1), _p(W2), _p(W3), _p(out), _p(mag))
    return (out, mag) if with_absmag else out


MLP_BF16, MLP_EXACT = 0, 1


def mlp_bwd(x, W1, W2, W3, d_y, mode: int = MLP_BF16, with_mag: bool = False):
    """Returns dict(d_x, dW1, dW2, dW3, margin) in binary64 (plus mag_d_x,
    mag_dW1..3 with ``with_mag``).  mode MLP_BF16: operands rounded to
    bfloat16 where the kernel feeds its matrix unit; MLP_EXACT: the
    network's derivative with no rounding beyond the stored activations."""
    x, W1, W2, W3 = _h(x), _h(W1), _h(W2), _h(W3)
    N, d_in = x.shape
    H, d_out = W1.shape[0], W3.shape[0]
    dy = np.ascontiguousarray(d_y, np.float32)
    assert dy.shape == (N, d_out)
    out = dict(d_x=np.zeros((N, d_in), np.float64), dW1=np.zeros((H, d_in), np.float64),
               dW2=np.zeros((H, H), np.float64), dW3=np.zeros((d_out, H), np.float64),
               margin=np.zeros(N, np.float64))
    mags = [None] * 4
    if with_mag:
        for k in ("d_x", "dW1", "dW2", "dW3"):
            out["mag_" + k] = np.zeros_like(out[k])
        mags = [out["mag_d_x"], out["mag_dW1"], out["mag_dW2"], out["mag_dW3"]]
    lib().orc_mlp_bwd(N, d_in, H, d_out, _p(x), _p(W1), _p(W2), _p(W3), _p(dy), int(mode), _p(out["d_x"]),
                      _p(out["dW1"]), _p(out["dW2"]), _p(out["dW3"]), _p(out["margin"]), *[_p(m) for m in mags])
    return out


# --- optimizer -------------------------------------------------------------------

def adam_step(param, grad, m, v, lr, beta1, beta2, eps, step):
    """One Adam step on copies of the binary32 state; returns
    (param, m, v, param_f16_bits)."""
    p = np.array(param, np.float32, copy=True)
    g = np.ascontiguousarray(grad, np.float32)
    mm = np.array(m, np.float32, copy=True)
    vv = np.array(v, np.float32, copy=True)
    h = np.zeros(p.shape, np.uint16)
    lib().orc_adam_step(p.size, _p(p), _p(g), _p(mm), _p(vv), lr, beta1, beta2, eps, step, _p(h))
    return p, mm, vv, h


def mse_grad(y, target, scale: float) -> np.ndarray:
    a = np.ascontiguousarray(y, np.float32)
    b = np.ascontiguousarray(target, np.float32)
    out = np.zeros(a.shape, np.float64)
    lib().orc_mse_grad(a.size, _p(a), _p(b), float(scale), _p(out))
    return out


def cast_f32_f16(src) -> np.ndarray:
    s = np.ascontiguousarray(src, np.float32)
    out = np.zeros(s.shape, np.uint16)
    lib().orc_cast_f32_f16(s.size, _p(s), _p(out))
    return out


def encode_input_grad(e: Encoding, pts, tables, d_out, with_mag: bool = False):
    """d L / d x [N, n] in binary64 for the output gradient d_out [N, L*F]."""
    x = _pts(pts, e.n_dims)
    t = _tables(e, tables)
    g = np.ascontiguousarray(d_out, np.float64)
    out = np.zeros((len(x), e.n_dims), np.float64)
    mag = np.zeros_like(out) if with_mag else None
    ce = e._c()
    lib().orc_encode_input_grad(C.byref(ce), len(x), _p(x), _p(t), _p(g), _p(out), _p(mag) if with_mag else None)
    return (out, mag) if with_mag else out


# --- volume rendering (Eq. 5) ---------------------------------------------------

def composite_fwd(raw, delta) -> np.ndarray:
    """raw [R, S, 4] float32 (density, colour before activation), delta
    [R, S] float32 -> rgba [R, 4] in binary64."""
    a = np.ascontiguousarray(raw, np.float32)
    d = np.ascontiguousarray(delta, np.float32)
    R, S = a.shape[0], a.shape[1]
    out = np.zeros((R, 4), np.float64)
    lib().orc_composite_fwd(R, S, _p(a), _p(d), _p(out))
    return out


def composite_bwd(raw, delta, d_rgba, with_mag: bool = False):
    """Adjoint: d_raw [R, S, 4] (and the magnitude bound terms)."""
    a = np.ascontiguousarray(raw, np.float32)
    d = np.ascontiguousarray(delta, np.float32)
    g = np.ascontiguousarray(d_rgba, np.float64)
    R, S = a.shape[0], a.shape[1]
    out = np.zeros((R, S, 4), np.float64)
    mag = np.zeros((R, S, 4), np.float64) if with_mag else None
    lib().orc_composite_bwd(R, S, _p(a), _p(d), _p(g), _p(out), _p(mag) if with_mag else None)
    return (out, mag) if with_mag else out


def set_threads(n: int) -> None:
    """OpenMP threads of the parallel oracle loops (for timing)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())

