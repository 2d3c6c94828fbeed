"""Python binding of libgrb (the C ABI declared in include/grb.h).

Argument marshalling only: torch supplies device memory and the HIP stream,
every computation runs in the library's HIP kernels.  Importing this package
on a machine where libgrb.so was not built raises ImportError; there is no
fallback path.

Low-level functions keep the C names (``grb_bfs``, ``grb_mxv``, ...) and take
raw pointers; the classes below (:class:`Matrix`, :class:`Vector`) and the
helpers (:func:`bfs`, :func:`sssp`, :func:`pagerank`, :func:`mxv`,
:func:`vxm`) wrap them around torch tensors.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrb.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_1908_01407_amd/build.py`")

# torch first: the library and torch both link the HIP runtime, and the one
# loaded first serves the process.  Loaded the other way round, torch's own
# kernels failed to launch ("invalid device function").
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# ---- enums and flags (mirror include/grb.h) ---------------------------------
GRB_SUCCESS = 0
ERRORS = {
    1: "GRB_NO_VALUE", 2: "GRB_UNINITIALIZED_OBJECT", 3: "GRB_NULL_POINTER",
    4: "GRB_INVALID_VALUE", 5: "GRB_INVALID_INDEX", 6: "GRB_DOMAIN_MISMATCH",
    7: "GRB_DIMENSION_MISMATCH", 8: "GRB_NOT_IMPLEMENTED", 9: "GRB_INSUFFICIENT_SPACE",
    10: "GRB_OUT_OF_MEMORY", 11: "GRB_PANIC",
}
GRB_BOOL, GRB_INT32, GRB_FP32, GRB_FP64 = 0, 1, 2, 3
SEMIRINGS = {
    "lor_land": 0, "min_plus_fp32": 1, "min_plus_fp64": 2, "plus_times_fp32": 3,
    "plus_times_fp64": 4, "min_first_int32": 5, "min_second_int32": 6, "plus_pair_int32": 7,
}
ACCUMS = {None: 0, "min": 1, "plus": 2, "lor": 3}
GRB_MASK_COMP, GRB_MASK_STRUCT, GRB_TRAN_A, GRB_REPLACE, GRB_PROFILE = 0x1, 0x2, 0x4, 0x8, 0x10
GRB_LOOP_NO_WAIT = 0x20  # test hook: the multi-workgroup loop gives up every barrier at once
DIR_AUTO, DIR_PUSH, DIR_PULL = 0, 1, 2
SWITCH_PAPER, SWITCH_EXACT = 0, 1
GRB_MATRIX_SYMMETRIC = 0x1
OP_MXV, OP_BFS, OP_SSSP, OP_PAGERANK, OP_MSBFS, OP_NVALS, OP_MXM, OP_EXTRACT, OP_CC = range(9)
STATS_MAX = 256


class GrbError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.grb_error_string(code).decode()
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({msg})")


class Descriptor(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("direction", ctypes.c_int32),
                ("switch_rule", ctypes.c_int32), ("switch_denominator", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class MsbfsTile(ctypes.Structure):
    _fields_ = [("words_per_pass", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class Stats(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("recorded", ctypes.c_int32), ("pushes", ctypes.c_int32),
                ("pulls", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("edges_push", ctypes.c_int64), ("expand_ms_push", ctypes.c_double),
                ("expand_ms_pull", ctypes.c_double), ("expand_ms_all", ctypes.c_double),
                ("direction", ctypes.c_int32 * STATS_MAX),
                ("frontier", ctypes.c_int64 * STATS_MAX),
                ("edges", ctypes.c_int64 * STATS_MAX),
                ("kernel_ms", ctypes.c_float * STATS_MAX)]


_p, _i32, _i64, _u32, _sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                             ctypes.c_size_t)
_PP = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "grb_version": ([], _i32),
    "grb_error_string": ([_i32], ctypes.c_char_p),
    "grb_descriptor_init": ([ctypes.POINTER(Descriptor)], _i32),
    "grb_last_stats": ([ctypes.POINTER(Stats)], _i32),
    "grb_stream_check": ([_p], _i32),
    "grb_csr_build": ([_PP, _i64, _i64, _p, _p, _p, ctypes.c_int], _i32),
    "grb_csr_nnz": ([_p, ctypes.POINTER(_i64)], _i32),
    "grb_csr_copy": ([_p, _p, _p, _p], _i32),
    "grb_csr_free": ([_PP], _i32),
    "grb_csr_lower_by_degree": ([_p, _PP, _p], _i32),
    "grb_mxm_masked": ([_p, _p, _p, _p, _i32, ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
    "grb_tricount": ([ctypes.POINTER(_i64), _p, ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
    "grb_matrix_create": ([_PP, _i64, _i64, _i64, _p, _p, _p, _i32, _p, _p, _p, _u32], _i32),
    "grb_matrix_free": ([_PP], _i32),
    "grb_matrix_nrows": ([_p, ctypes.POINTER(_i64)], _i32),
    "grb_matrix_ncols": ([_p, ctypes.POINTER(_i64)], _i32),
    "grb_matrix_nvals": ([_p, ctypes.POINTER(_i64)], _i32),
    "grb_matrix_meta_size": ([_p, ctypes.POINTER(_sz)], _i32),
    "grb_matrix_prepare": ([_p, _p, _sz, _p], _i32),
    "grb_vector_create": ([_PP, _i64, _i32, _p, _p, _p, _p], _i32),
    "grb_vector_free": ([_PP], _i32),
    "grb_vector_size": ([_p, ctypes.POINTER(_i64)], _i32),
    "grb_vector_clear": ([_p, _p], _i32),
    "grb_vector_fill": ([_p, _p, _p], _i32),
    "grb_vector_build": ([_p, _p, _p, _i64, _p], _i32),
    "grb_vector_nvals": ([_p, ctypes.POINTER(_i64), _p, _sz, _p], _i32),
    "grb_vector_extract": ([_p, _p, _p, _i64, ctypes.POINTER(_i64), _p, _sz, _p], _i32),
    "grb_workspace_size": ([_i32, _p, _i64, ctypes.POINTER(_sz)], _i32),
    "grb_mxv": ([_p, _p, _i32, _i32, _p, _p, ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
    "grb_vxm": ([_p, _p, _i32, _i32, _p, _p, ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
    "grb_bfs": ([_p, _p, _p, _i32, ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
    "grb_sssp": ([_p, _p, _i32, ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
    "grb_sssp_delta": ([_p, _p, _i32, ctypes.c_float, ctypes.POINTER(Descriptor), _p, _sz, _p],
                       _i32),
    "grb_msbfs": ([_p, _p, _p, _i32, ctypes.POINTER(MsbfsTile), ctypes.POINTER(Descriptor), _p,
                   _sz, _p], _i32),
    "grb_msbfs_session_create": ([_PP, _p, _i32, _p, ctypes.POINTER(MsbfsTile),
                                  ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
    "grb_msbfs_session_join": ([_p, _p, _p, _i32, _p], _i32),
    "grb_msbfs_session_step": ([_p, _i32, _p, ctypes.POINTER(_i32), _p], _i32),
    "grb_msbfs_session_extract": ([_p, _p, _i32, _p, _p], _i32),
    "grb_msbfs_session_free": ([_PP], _i32),
    "grb_bfs_noalloc": ([_p, _p, _p, _i32, ctypes.POINTER(Descriptor), _p], _i32),
    "grb_cc": ([_p, _p, ctypes.POINTER(_i32), ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
    "grb_pagerank": ([_p, _i32, _p, ctypes.c_double, _i32, ctypes.c_double,
                      ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_double),
                      ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
    "grb_pagerank_adaptive": ([_p, _i32, _p, ctypes.c_double, _i32, ctypes.c_double,
                               ctypes.c_double, ctypes.POINTER(_i32),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(Descriptor), _p, _sz, _p], _i32),
}

#: every C symbol this binding exposes, with its ctypes function
C_FUNCTIONS = {}
for _name, (_args, _ret) in _SIGS.items():
    _f = getattr(_lib, _name, None)
    if _f is None:
        continue
    _f.argtypes = _args
    _f.restype = _ret
    C_FUNCTIONS[_name] = _f
    globals()[_name] = _f


def check(code: int, where: str = "grb") -> None:
    if code != GRB_SUCCESS:
        raise GrbError(code, where)


def descriptor(*, direction: int = DIR_AUTO, rule: int = SWITCH_PAPER, denominator: int = 10,
               flags: int = 0, max_iter: int = 0) -> Descriptor:
    d = Descriptor()
    check(_lib.grb_descriptor_init(ctypes.byref(d)), "grb_descriptor_init")
    d.flags = flags
    d.direction = direction
    d.switch_rule = rule
    d.switch_denominator = denominator
    d.max_iter = max_iter
    return d


def last_stats() -> dict:
    s = Stats()
    check(_lib.grb_last_stats(ctypes.byref(s)), "grb_last_stats")
    r = s.recorded
    return {
        "op": s.op, "iterations": s.iterations, "pushes": s.pushes, "pulls": s.pulls,
        "edges_push": s.edges_push, "expand_ms_push": s.expand_ms_push,
        "expand_ms_pull": s.expand_ms_pull, "launches": s.launches,
        "expand_ms_all": s.expand_ms_all,
        "direction": list(s.direction[:r]), "frontier": list(s.frontier[:r]),
        "edges": list(s.edges[:r]), "kernel_ms": list(s.kernel_ms[:r]),
    }


# ---- host CSR construction ---------------------------------------------------

def csr_from_edges(n: int, src, dst, w=None, symmetrise: bool = True):
    """Cleaned CSR (row_ptr, col_idx, values or None) as numpy arrays."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
        wp = w.ctypes.data
    h = ctypes.c_void_p()
    check(_lib.grb_csr_build(ctypes.byref(h), n, src.shape[0], src.ctypes.data, dst.ctypes.data,
                             wp, 1 if symmetrise else 0), "grb_csr_build")
    try:
        nnz = ctypes.c_int64()
        check(_lib.grb_csr_nnz(h, ctypes.byref(nnz)), "grb_csr_nnz")
        rp = np.empty(n + 1, dtype=np.int32)
        ci = np.empty(max(nnz.value, 0), dtype=np.int32)
        vals = np.empty(nnz.value, dtype=np.float32) if w is not None else None
        check(_lib.grb_csr_copy(h, rp.ctypes.data, ci.ctypes.data if nnz.value else None,
                                vals.ctypes.data if vals is not None and nnz.value else None),
              "grb_csr_copy")
    finally:
        _lib.grb_csr_free(ctypes.byref(h))
    return rp, ci, vals


def _csr_out(h, n):
    nnz = ctypes.c_int64()
    check(_lib.grb_csr_nnz(h, ctypes.byref(nnz)), "grb_csr_nnz")
    rp = np.empty(n + 1, dtype=np.int32)
    ci = np.empty(max(nnz.value, 0), dtype=np.int32)
    check(_lib.grb_csr_copy(h, rp.ctypes.data, ci.ctypes.data if nnz.value else None, None),
          "grb_csr_copy")
    return rp, ci


def lower_by_degree(n: int, src, dst):
    """Triangle-counting input via grb_csr_lower_by_degree: the symmetrised,
    cleaned graph renumbered by decreasing degree, strict lower triangle.
    Returns (row_ptr, col_idx, rank) as numpy arrays."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    h = ctypes.c_void_p()
    lo = ctypes.c_void_p()
    check(_lib.grb_csr_build(ctypes.byref(h), n, src.shape[0], src.ctypes.data, dst.ctypes.data,
                             None, 1), "grb_csr_build")
    try:
        rank = np.empty(max(n, 1), dtype=np.int32)
        check(_lib.grb_csr_lower_by_degree(h, ctypes.byref(lo), rank.ctypes.data),
              "grb_csr_lower_by_degree")
        try:
            rp, ci = _csr_out(lo, n)
        finally:
            _lib.grb_csr_free(ctypes.byref(lo))
    finally:
        _lib.grb_csr_free(ctypes.byref(h))
    return rp, ci, rank[:n]


# ---- torch-backed objects ---------------------------------------------------------

def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    torch = _torch()
    # the current stream's raw handle without building a Stream object
    # (about 3 us per call that way); the public call where torch lacks it
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(raw(torch.cuda.current_device()))


def workspace(op: int, A: "Matrix", k: int = 0, device=None):
    torch = _torch()
    n = ctypes.c_size_t()
    check(_lib.grb_workspace_size(op, A.handle if A is not None else None, k, ctypes.byref(n)),
          "grb_workspace_size")
    dev = device if device is not None else (A.device if A is not None else "cuda")
    return torch.empty(max(n.value, 256), dtype=torch.uint8, device=dev)


class Matrix:
    """Device CSR (plus optional CSR of the transpose) wrapped in a grb_matrix."""

    def __init__(self, n_rows, n_cols, row_ptr, col_idx, values=None, t_row_ptr=None,
                 t_col_idx=None, t_values=None, symmetric=False, device="cuda", stream=None):
        torch = _torch()
        dev = torch.device(device)
        self.device = dev

        def to_dev(a, dt):
            if a is None:
                return None
            if isinstance(a, np.ndarray):
                a = torch.from_numpy(np.ascontiguousarray(a))
            if a.numel() == 0:  # keep a valid (non-null) device address
                return torch.zeros(1, dtype=dt, device=dev)
            return a.to(device=dev, dtype=dt).contiguous()

        self.row_ptr = to_dev(row_ptr, torch.int32)
        self.col_idx = to_dev(col_idx, torch.int32)
        vdt = torch.float64 if (values is not None and getattr(values, "dtype", None) in
                                (np.float64, torch.float64)) else torch.float32
        self.values = to_dev(values, vdt)
        self.t_row_ptr = to_dev(t_row_ptr, torch.int32)
        self.t_col_idx = to_dev(t_col_idx, torch.int32)
        self.t_values = to_dev(t_values, vdt)
        self.nrows, self.ncols = int(n_rows), int(n_cols)
        self.nnz = int(col_idx.shape[0]) if hasattr(col_idx, "shape") else len(col_idx)
        vtype = GRB_FP64 if vdt == torch.float64 else GRB_FP32
        h = ctypes.c_void_p()
        check(_lib.grb_matrix_create(
            ctypes.byref(h), self.nrows, self.ncols, self.nnz, _ptr(self.row_ptr),
            _ptr(self.col_idx) if self.nnz else None, _ptr(self.values), vtype,
            _ptr(self.t_row_ptr), _ptr(self.t_col_idx) if self.t_row_ptr is not None and self.nnz
            else None, _ptr(self.t_values), GRB_MATRIX_SYMMETRIC if symmetric else 0),
            "grb_matrix_create")
        self.handle = h
        sz = ctypes.c_size_t()
        check(_lib.grb_matrix_meta_size(h, ctypes.byref(sz)), "grb_matrix_meta_size")
        self.meta = torch.empty(max(sz.value, 256), dtype=torch.uint8, device=dev)
        check(_lib.grb_matrix_prepare(h, _ptr(self.meta), self.meta.numel(), _stream(stream)),
              "grb_matrix_prepare")

    @classmethod
    def from_raw(cls, g, device="cuda", weights=True, transpose=True):
        """From a graphgen.RawGraph: symmetric graphs share one CSR; directed
        graphs also get the CSR of the transpose (built from swapped edges)."""
        w = g.w if weights else None
        rp, ci, vals = csr_from_edges(g.n, g.src, g.dst, w, symmetrise=g.symmetric)
        if g.symmetric:
            return cls(g.n, g.n, rp, ci, vals, symmetric=True, device=device)
        trp = tci = tvals = None
        if transpose:
            trp, tci, tvals = csr_from_edges(g.n, g.dst, g.src, w, symmetrise=False)
        return cls(g.n, g.n, rp, ci, vals, trp, tci, tvals, symmetric=False, device=device)

    def __del__(self):
        h = getattr(self, "handle", None)
        try:
            if h is not None and h.value:
                _lib.grb_matrix_free(ctypes.byref(h))
        except (AttributeError, TypeError):
            pass  # module globals already torn down at interpreter exit


_TYPE_OF = {}


def _type_code(dtype):
    torch = _torch()
    return {torch.uint8: GRB_BOOL, torch.bool: GRB_BOOL, torch.int32: GRB_INT32,
            torch.float32: GRB_FP32, torch.float64: GRB_FP64}[dtype]


class Vector:
    """A grb_vector over device tensors: `values` [n] (or None: every entry is
    1), the presence `bitmap` [(n+63)/64] (dense form, or None), and the
    sparse form's sorted `indices` [n] with their device `count` [1] (or
    None).  At least one of the two forms."""

    def __init__(self, n: int, dtype=None, device="cuda", *, dense: bool = True,
                 sparse: bool = False, values: bool = True):
        torch = _torch()
        if not (dense or sparse):
            raise ValueError("Vector: needs the dense (bitmap) or the sparse (list) form")
        dtype = dtype if dtype is not None else torch.float32
        if dtype == torch.bool:
            dtype = torch.uint8
        self.n = int(n)
        self.dtype = dtype
        self.values = torch.zeros(max(self.n, 1), dtype=dtype, device=device) if values else None
        self.bitmap = (torch.zeros(max((self.n + 63) // 64, 1), dtype=torch.int64, device=device)
                       if dense else None)
        self.indices = torch.zeros(max(self.n, 1), dtype=torch.int32, device=device) if sparse \
            else None
        self.count = torch.zeros(1, dtype=torch.int32, device=device) if sparse else None
        h = ctypes.c_void_p()
        check(_lib.grb_vector_create(ctypes.byref(h), self.n, _type_code(dtype), _ptr(self.values),
                                     _ptr(self.bitmap), _ptr(self.indices), _ptr(self.count)),
              "grb_vector_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        try:
            if h is not None and h.value:
                _lib.grb_vector_free(ctypes.byref(h))
        except (AttributeError, TypeError):
            pass  # module globals already torn down at interpreter exit

    @property
    def device(self):
        for t in (self.values, self.bitmap, self.indices):
            if t is not None:
                return t.device
        return None

    def set(self, entries: dict, stream=None):
        """Clears, then sets the given {index: value} entries (via
        grb_vector_build; a vector without values takes the indices only)."""
        torch = _torch()
        keys = sorted(entries)
        idx = torch.tensor(keys, dtype=torch.int32, device=self.device)
        vals = None
        if self.values is not None:
            vals = torch.tensor([entries[i] for i in keys], dtype=self.dtype, device=self.device)
        check(_lib.grb_vector_build(self.handle, _ptr(idx) if idx.numel() else None,
                                    _ptr(vals) if vals is not None and vals.numel() else None,
                                    idx.numel(), _stream(stream)), "grb_vector_build")
        torch.cuda.current_stream().synchronize()

    def set_list(self, entries: dict):
        """Writes the sparse form directly, as its owner (sorted indices,
        count and values; the bitmap too when the vector has one)."""
        torch = _torch()
        keys = sorted(entries)
        if self.indices is None:
            raise ValueError("set_list: the vector has no list")
        if keys:
            self.indices[: len(keys)] = torch.tensor(keys, dtype=torch.int32, device=self.device)
            if self.values is not None:
                self.values.zero_()
                self.values[torch.tensor(keys, dtype=torch.int64, device=self.device)] = \
                    torch.tensor([entries[i] for i in keys], dtype=self.dtype, device=self.device)
        self.count.fill_(len(keys))
        if self.bitmap is not None:
            bits = np.zeros(self.bitmap.numel() * 64, dtype=np.uint8)
            bits[keys] = 1
            words = np.packbits(bits, bitorder="little").view(np.int64)
            self.bitmap.copy_(torch.from_numpy(words))
        torch.cuda.current_stream().synchronize()

    def set_any(self, entries: dict):
        """set() for a vector with a bitmap, set_list() for a list-only one."""
        if self.bitmap is not None:
            self.set(entries)
        else:
            self.set_list(entries)

    def fill(self, value=None, stream=None):
        """Every index present with `value` (grb_vector_fill)."""
        torch = _torch()
        buf = None
        if self.values is not None:
            buf = np.array([value], dtype=torch.empty(0, dtype=self.dtype).numpy().dtype)
        check(_lib.grb_vector_fill(self.handle, buf.ctypes.data if buf is not None else None,
                                   _stream(stream)), "grb_vector_fill")
        torch.cuda.current_stream().synchronize()

    def clear(self, stream=None):
        check(_lib.grb_vector_clear(self.handle, _stream(stream)), "grb_vector_clear")
        _torch().cuda.current_stream().synchronize()

    def extract_code(self, capacity=None, ws=None, stream=None):
        """(grb_info, nvals) of grb_vector_extract into host buffers of
        `capacity` entries (default n); the tuples are kept in
        self._extracted when the call succeeds."""
        torch = _torch()
        cap = self.n if capacity is None else int(capacity)
        idx = np.zeros(max(cap, 1), dtype=np.int32)
        vals = np.zeros(max(cap, 1), dtype=torch.empty(0, dtype=self.dtype).numpy().dtype)
        ws = ws if ws is not None else workspace(OP_EXTRACT, None, self.n, device=self.device)
        nv = ctypes.c_int64()
        code = _lib.grb_vector_extract(self.handle, idx.ctypes.data, vals.ctypes.data, cap,
                                       ctypes.byref(nv), _ptr(ws), ws.numel(), _stream(stream))
        if code == GRB_SUCCESS:
            self._extracted = (idx[: nv.value].copy(), vals[: nv.value].copy())
        return code, nv.value

    def extract(self, ws=None, stream=None):
        """(indices int32[k], values[k]) of the present entries, ascending,
        via grb_vector_extract."""
        code, _ = self.extract_code(None, ws, stream)
        check(code, "grb_vector_extract")
        return self._extracted

    def to_dict(self) -> dict:
        """Present entries as {index: value}, read straight from the device
        arrays (the bitmap, else the list)."""
        torch = _torch()
        if self.bitmap is not None:
            bm = self.bitmap.cpu().numpy().view(np.uint64)
            bits = np.unpackbits(bm.view(np.uint8), bitorder="little")[: self.n].astype(bool)
            present = np.flatnonzero(bits)
        else:
            c = int(self.count.cpu()[0])
            present = self.indices[:c].cpu().numpy()
        vals = self.values.cpu().numpy() if self.values is not None else None
        out = {}
        for i in present:
            if vals is None:
                out[int(i)] = True if self.dtype == torch.uint8 else 1
                continue
            v = vals[i]
            out[int(i)] = bool(v) if self.dtype == torch.uint8 else v.item()
        return out


# ---- drivers and products --------------------------------------------------------

def bfs(A: Matrix, source: int, *, parents: bool = True, desc: Descriptor | None = None,
        ws=None, stream=None, out=None):
    """(levels int32[n], parents int32[n] or None) via grb_bfs.  `out` may
    pass (levels, parents) device tensors of at least n entries to fill."""
    torch = _torch()
    if out is not None:
        lev, par = out
        if lev.numel() < A.nrows or (parents and (par is None or par.numel() < A.nrows)):
            raise ValueError("bfs: output tensors hold fewer than n entries")
        if not parents:
            par = None
    else:
        lev = torch.empty(max(A.nrows, 1), dtype=torch.int32, device=A.device)
        par = torch.empty(max(A.nrows, 1), dtype=torch.int32, device=A.device) if parents else None
    ws = ws if ws is not None else workspace(OP_BFS, A)
    check(_lib.grb_bfs(_ptr(lev), _ptr(par), A.handle, int(source),
                       ctypes.byref(desc) if desc is not None else None, _ptr(ws), ws.numel(),
                       _stream(stream)), "grb_bfs")
    n = A.nrows  # views only where the buffers are longer than n
    return (lev if lev.numel() == n else lev[:n]), \
        (par if par is None or par.numel() == n else par[:n])


def sssp(A: Matrix, source: int, *, delta: float | None = None, desc: Descriptor | None = None,
         ws=None, stream=None):
    """dist fp32[n] via grb_sssp, or via grb_sssp_delta when `delta` (the
    bucket width) is given."""
    torch = _torch()
    dist = torch.empty(max(A.nrows, 1), dtype=torch.float32, device=A.device)
    ws = ws if ws is not None else workspace(OP_SSSP, A)
    dp = ctypes.byref(desc) if desc is not None else None
    if delta is None:
        check(_lib.grb_sssp(_ptr(dist), A.handle, int(source), dp, _ptr(ws), ws.numel(),
                            _stream(stream)), "grb_sssp")
    else:
        check(_lib.grb_sssp_delta(_ptr(dist), A.handle, int(source), float(delta), dp, _ptr(ws),
                                  ws.numel(), _stream(stream)), "grb_sssp_delta")
    return dist[: A.nrows]


def msbfs(A: Matrix, sources, *, words_per_pass: int = 0, grid: int = 0,
          desc: Descriptor | None = None, ws=None, levels=None, stream=None):
    """levels int32[n, k] (vertex-major) of k BFS runs via grb_msbfs."""
    torch = _torch()
    if not isinstance(sources, torch.Tensor):
        sources = torch.as_tensor(np.asarray(sources, dtype=np.int32))
    src = sources.to(device=A.device, dtype=torch.int32).contiguous()
    k = int(src.numel())
    if levels is None:
        levels = torch.empty((max(A.nrows, 1), k), dtype=torch.int32, device=A.device)
    ws = ws if ws is not None else workspace(OP_MSBFS, A, k)
    tile = MsbfsTile(words_per_pass, grid)
    check(_lib.grb_msbfs(_ptr(levels), A.handle, _ptr(src), k, ctypes.byref(tile),
                         ctypes.byref(desc) if desc is not None else None, _ptr(ws), ws.numel(),
                         _stream(stream)), "grb_msbfs")
    return levels[: A.nrows]


class MsbfsSession:
    """Continuous batching of BFS queries on one graph (grb_msbfs_session_*):
    k lanes; queries join free lanes and retire at level boundaries while
    the others keep running.  All calls go to one stream."""

    def __init__(self, A: Matrix, k: int, *, words_per_pass: int = 0, grid: int = 0,
                 desc: Descriptor | None = None, ws=None, levels=None, stream=None):
        torch = _torch()
        self.A, self.k, self.n = A, int(k), A.nrows
        self.W = (self.k + 63) // 64
        self.stream = stream
        self.levels = levels if levels is not None else torch.empty(
            (max(A.nrows, 1), self.k), dtype=torch.int32, device=A.device)
        self.ws = ws if ws is not None else workspace(OP_MSBFS, A, self.k)
        tile = MsbfsTile(words_per_pass, grid)
        h = ctypes.c_void_p()
        check(_lib.grb_msbfs_session_create(
            ctypes.byref(h), A.handle, self.k, _ptr(self.levels), ctypes.byref(tile),
            ctypes.byref(desc) if desc is not None else None, _ptr(self.ws), self.ws.numel(),
            _stream(stream)), "grb_msbfs_session_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        try:
            if h is not None and h.value:
                _lib.grb_msbfs_session_free(ctypes.byref(h))
        except (AttributeError, TypeError):
            pass

    def join(self, lanes, sources):
        """Starts sources[i] in lane lanes[i] at the current level boundary."""
        ln = np.ascontiguousarray(lanes, dtype=np.int32)
        sr = np.ascontiguousarray(sources, dtype=np.int32)
        if ln.shape != sr.shape:
            raise ValueError("join: lanes and sources differ in length")
        check(_lib.grb_msbfs_session_join(self.handle, ln.ctypes.data, sr.ctypes.data, ln.size,
                                          _stream(self.stream)), "grb_msbfs_session_join")

    def step(self, max_levels: int):
        """Runs up to max_levels levels; returns (lanes that ended, levels run)."""
        done = np.zeros(self.W, dtype=np.uint64)
        ran = ctypes.c_int32()
        check(_lib.grb_msbfs_session_step(self.handle, int(max_levels), done.ctypes.data,
                                          ctypes.byref(ran), _stream(self.stream)),
              "grb_msbfs_session_step")
        bits = np.unpackbits(done.view(np.uint8), bitorder="little")[: self.k]
        return [int(q) for q in np.flatnonzero(bits)], ran.value

    def extract(self, lanes, out=None):
        """int32 [len(lanes), n] levels of the given lanes (-1 unreached)."""
        torch = _torch()
        ln = np.ascontiguousarray(lanes, dtype=np.int32)
        if out is None:
            out = torch.empty((max(ln.size, 1), max(self.n, 1)), dtype=torch.int32,
                              device=self.levels.device)
        check(_lib.grb_msbfs_session_extract(self.handle, ln.ctypes.data, ln.size, _ptr(out),
                                             _stream(self.stream)), "grb_msbfs_session_extract")
        return out[: ln.size, : self.n]


def cc(A: Matrix, *, desc: Descriptor | None = None, ws=None, stream=None):
    """(labels int32[n], iterations) via grb_cc: each vertex labelled with the
    smallest vertex id of its component."""
    torch = _torch()
    labels = torch.empty(max(A.nrows, 1), dtype=torch.int32, device=A.device)
    ws = ws if ws is not None else workspace(OP_CC, A)
    it = ctypes.c_int32()
    check(_lib.grb_cc(_ptr(labels), A.handle, ctypes.byref(it),
                      ctypes.byref(desc) if desc is not None else None, _ptr(ws), ws.numel(),
                      _stream(stream)), "grb_cc")
    return labels[: A.nrows], it.value


def pagerank(A: Matrix, *, dtype=None, damping: float = 0.85, max_iter: int = 50,
             tol: float = 1e-7, desc: Descriptor | None = None, ws=None, stream=None):
    """(p[n], iterations, last L1 delta) via grb_pagerank."""
    torch = _torch()
    dtype = dtype if dtype is not None else torch.float32
    t = GRB_FP64 if dtype == torch.float64 else GRB_FP32
    p = torch.empty(max(A.nrows, 1), dtype=dtype, device=A.device)
    ws = ws if ws is not None else workspace(OP_PAGERANK, A, 2 if t == GRB_FP64 else 1)
    iters = ctypes.c_int32()
    delta = ctypes.c_double()
    check(_lib.grb_pagerank(_ptr(p), t, A.handle, float(damping), int(max_iter), float(tol),
                            ctypes.byref(iters), ctypes.byref(delta),
                            ctypes.byref(desc) if desc is not None else None, _ptr(ws),
                            ws.numel(), _stream(stream)), "grb_pagerank")
    return p[: A.nrows], iters.value, delta.value


def pagerank_adaptive(A: Matrix, eps: float, *, dtype=None, damping: float = 0.85,
                      max_iter: int = 50, tol: float = 1e-7, desc: Descriptor | None = None,
                      ws=None, stream=None):
    """(p[n], iterations, last L1 delta, vertices still active) via
    grb_pagerank_adaptive (converged vertices frozen once their relative
    change is at most eps)."""
    torch = _torch()
    dtype = dtype if dtype is not None else torch.float32
    t = GRB_FP64 if dtype == torch.float64 else GRB_FP32
    p = torch.empty(max(A.nrows, 1), dtype=dtype, device=A.device)
    ws = ws if ws is not None else workspace(OP_PAGERANK, A, 2 if t == GRB_FP64 else 1)
    iters = ctypes.c_int32()
    delta = ctypes.c_double()
    active = ctypes.c_int64()
    check(_lib.grb_pagerank_adaptive(_ptr(p), t, A.handle, float(damping), int(max_iter),
                                     float(tol), float(eps), ctypes.byref(iters),
                                     ctypes.byref(delta), ctypes.byref(active),
                                     ctypes.byref(desc) if desc is not None else None, _ptr(ws),
                                     ws.numel(), _stream(stream)), "grb_pagerank_adaptive")
    return p[: A.nrows], iters.value, delta.value, active.value


def mxm_masked(M: Matrix, A: Matrix, B: Matrix, semiring: str = "plus_pair_int32", *,
               desc: Descriptor | None = None, ws=None, stream=None):
    """C = (A B^T) .* M via grb_mxm_masked: one value per entry of M, in M's
    CSR order (int32 for plus_pair_int32, float / double for plus_times)."""
    torch = _torch()
    dt = {"plus_pair_int32": torch.int32, "plus_times_fp32": torch.float32,
          "plus_times_fp64": torch.float64}.get(semiring, torch.int32)
    c = torch.empty(max(M.nnz, 1), dtype=dt, device=M.device)
    ws = ws if ws is not None else workspace(OP_MXM, None, device=M.device)
    check(_lib.grb_mxm_masked(_ptr(c), M.handle, A.handle, B.handle, SEMIRINGS[semiring],
                              ctypes.byref(desc) if desc is not None else None, _ptr(ws),
                              ws.numel(), _stream(stream)), "grb_mxm_masked")
    return c[: M.nnz]


def tricount(L: Matrix, *, desc: Descriptor | None = None, ws=None, stream=None) -> int:
    """Sum of (L L^T) .* L via grb_tricount: the triangle count when L is a
    strict lower triangle of a symmetric graph (see lower_by_degree)."""
    ws = ws if ws is not None else workspace(OP_MXM, None, device=L.device)
    out = ctypes.c_int64()
    check(_lib.grb_tricount(ctypes.byref(out), L.handle,
                            ctypes.byref(desc) if desc is not None else None, _ptr(ws),
                            ws.numel(), _stream(stream)), "grb_tricount")
    return out.value


def mxv(w: Vector, mask: Vector | None, accum, semiring: str, A: Matrix, u: Vector, *,
        desc: Descriptor | None = None, ws=None, stream=None):
    ws = ws if ws is not None else workspace(OP_MXV, A)
    check(_lib.grb_mxv(w.handle, mask.handle if mask is not None else None, ACCUMS[accum],
                       SEMIRINGS[semiring], A.handle, u.handle,
                       ctypes.byref(desc) if desc is not None else None, _ptr(ws), ws.numel(),
                       _stream(stream)), "grb_mxv")


def vxm(w: Vector, mask: Vector | None, accum, semiring: str, u: Vector, A: Matrix, *,
        desc: Descriptor | None = None, ws=None, stream=None):
    ws = ws if ws is not None else workspace(OP_MXV, A)
    check(_lib.grb_vxm(w.handle, mask.handle if mask is not None else None, ACCUMS[accum],
                       SEMIRINGS[semiring], u.handle, A.handle,
                       ctypes.byref(desc) if desc is not None else None, _ptr(ws), ws.numel(),
                       _stream(stream)), "grb_vxm")
