"""ctypes binding of libpk.so: the same entry points as include/pk.h.

Argument marshalling only -- every step of the path runs in the library and
its HIP kernels.  Matrices may be passed as torch tensors (device memory);
their data pointers, leading dimensions and the current HIP stream are
forwarded.  Calls raise if the library has not been built.

HIP runtime: libpk.so links the HIP runtime of the ROCm it was built with;
PyTorch wheels bundle their own copy under the same soname.  The library is
opened after torch is imported, so it binds to the runtime torch already
loaded and one runtime serves the process (stream handles and device
pointers are shared).  The machine parameters the case table binds are the
ones that runtime reports: in a process with torch 2.10's bundled ROCm 7.0
runtime gfx950 reports 65536 registers per workgroup, the system ROCm 7.2
runtime alone reports 131072.
"""
from __future__ import annotations

import ctypes
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpk.so")

PK_OK = 0
PK_ERR_INVALID_ARG = -1
PK_ERR_NO_FEASIBLE_BRANCH = -2
PK_ERR_UNSUPPORTED_DTYPE = -3
PK_ERR_NOT_INSTANTIATED = -4
PK_ERR_HIP = -5
PK_ERR_COST_MODEL = -6
PK_ERR_BUFFER_TOO_SMALL = -7
PK_ERR_PARSE = -8

PK_F32, PK_I32, PK_BF16 = 0, 1, 2
PK_FAMILY_VALU, PK_FAMILY_MFMA, PK_FAMILY_TRANSPOSE, PK_FAMILY_MADD, PK_FAMILY_JACOBI, PK_FAMILY_POLYDIV = (
    0, 1, 2, 3, 4, 5)
PK_FAMILY_VALU2 = 6
PK_VALU_GRAN, PK_VALU_NOLDS = 1, 2
PK_POLYDIV_FUSED, PK_POLYDIV_WIDE = 4, 8
PK_JACOBI_FUSED = 4
PK_MFMA_SINGLE = 1
PK_MFMA_SPLIT = 16  # internal: the form of a program that runs shares of K
PK_POLICY_CASE, PK_POLICY_LEARNED, PK_POLICY_EXHAUSTIVE = 0, 1, 2

DTYPES = {"f32": PK_F32, "i32": PK_I32, "bf16": PK_BF16}


class PkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("pk error %d: %s" % (code, msg))
        self.code = code


class pk_machine(ctypes.Structure):
    _fields_ = [("wave", ctypes.c_int32), ("lds_block", ctypes.c_int64), ("lds_cu", ctypes.c_int64),
                ("regs_block", ctypes.c_int64), ("regs_cu", ctypes.c_int64),
                ("max_threads_block", ctypes.c_int32), ("max_threads_cu", ctypes.c_int32),
                ("max_blocks_cu", ctypes.c_int32), ("cu_count", ctypes.c_int32),
                ("clock_khz", ctypes.c_int32), ("arch", ctypes.c_char * 64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["arch"] = self.arch.decode()
        return d


class pk_params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("family", "leaf", "variant", "bx", "by", "s", "bk", "bm", "bn", "wm", "wn", "ks", "sy")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    def __repr__(self):
        return "pk_params(%s)" % ", ".join("%s=%d" % kv for kv in self.as_dict().items())


def params(family=PK_FAMILY_VALU, leaf=-1, variant=-1, bx=0, by=0, s=0, bk=0, bm=0, bn=0, wm=0, wn=0, ks=0, sy=0):
    return pk_params(family, leaf, variant, bx, by, s, bk, bm, bn, wm, wn, ks, sy)


def machine(**kw) -> pk_machine:
    m = pk_machine()
    for k, v in kw.items():
        if k == "arch":
            m.arch = v.encode() if isinstance(v, str) else v
        else:
            setattr(m, k, v)
    return m


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpk.so is not built; run __graft_entry__.build() (or python -m "
                               "paper_1801_04348_amd.build)")
        try:  # torch first: the library then binds to torch's HIP runtime
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
        L.pk_last_error.restype = ctypes.c_char_p
        L.pk_version.restype = ctypes.c_char_p
        L.pk_instance_count.restype = i32
        L.pk_instance_name.restype = ctypes.c_char_p
        L.pk_instance_name.argtypes = [i32]
        L.pk_machine_query.argtypes = [i32, ctypes.POINTER(pk_machine)]
        L.pk_co_solve.argtypes = [ctypes.c_char_p, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
        L.pk_case_table_build.argtypes = [i32, ctypes.POINTER(pk_machine), ctypes.POINTER(vp)]
        L.pk_case_table_free.argtypes = [vp]
        L.pk_case_table_free.restype = None
        L.pk_case_table_describe.argtypes = [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
        L.pk_case_table_lookup.argtypes = [vp, i32, ctypes.POINTER(pk_params), ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)]
        L.pk_select.argtypes = [vp, i32, i64, i64, i64, i32, ctypes.POINTER(pk_params)]
        L.pk_matmul.argtypes = [vp, ctypes.POINTER(pk_params), i32, vp, i64, vp, i64, vp, i64, i64, i64, i64,
                                i32, vp]
        L.pk_launch_shape.argtypes = [vp, ctypes.POINTER(pk_params), i32, i64, i64, i64,
                                      ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(i64)]
        L.pk_select_operands.argtypes = [vp, i32, vp, i64, vp, i64, i64, i64, i64, i32, ctypes.POINTER(pk_params)]
        L.pk_select_operands.restype = i32
        L.pk_measure.argtypes = [vp, i32, vp, i64, vp, i64, vp, i64, i64, i64, i64, ctypes.POINTER(pk_params),
                                 ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(ctypes.c_int)]
        L.pk_transpose.argtypes = [vp, ctypes.POINTER(pk_params), i32, vp, i64, vp, i64, i64, i64, vp]
        L.pk_transpose.restype = i32
        L.pk_select_transpose.argtypes = [vp, i32, i64, i64, i32, ctypes.POINTER(pk_params)]
        L.pk_select_transpose.restype = i32
        L.pk_probe_valu_rate.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
        L.pk_probe_valu_rate.restype = i32
        L.pk_estimate.argtypes = [vp, ctypes.POINTER(pk_params), i32, i64, i64, i64, i32,
                                  ctypes.POINTER(ctypes.c_double)]
        L.pk_estimate.restype = i32
        L.pk_madd.argtypes = [vp, ctypes.POINTER(pk_params), i32, vp, i64, vp, i64, vp, i64, i64, i64, vp]
        L.pk_madd.restype = i32
        L.pk_select_madd.argtypes = [vp, i32, i64, i64, i32, ctypes.POINTER(pk_params)]
        L.pk_select_madd.restype = i32
        L.pk_jacobi1d.argtypes = [vp, ctypes.POINTER(pk_params), i32, vp, i64, i64, vp]
        L.pk_jacobi1d.restype = i32
        L.pk_select_jacobi1d.argtypes = [vp, i32, i64, i64, i32, ctypes.POINTER(pk_params)]
        L.pk_select_jacobi1d.restype = i32
        L.pk_polydiv.argtypes = [vp, ctypes.POINTER(pk_params), vp, i64, vp, i64, ctypes.c_uint32, vp]
        L.pk_polydiv.restype = i32
        L.pk_select_polydiv.argtypes = [vp, i64, i64, i32, ctypes.POINTER(pk_params)]
        L.pk_select_polydiv.restype = i32
        L.pk_kernel_name.argtypes = [vp, ctypes.POINTER(pk_params), i32]
        L.pk_kernel_name.restype = ctypes.c_char_p
        f32p = ctypes.POINTER(ctypes.c_float)
        L.pk_features.argtypes = [vp, ctypes.POINTER(pk_params), i32, i64, i64, i64, i32, f32p]
        L.pk_costmodel_train.argtypes = [vp, f32p, f32p, i64, i32, ctypes.c_float, ctypes.c_uint64,
                                         ctypes.POINTER(vp), f32p]
        L.pk_costmodel_predict.argtypes = [vp, i32, f32p, i64, f32p]
        L.pk_costmodel_grad.argtypes = [i32, f32p, f32p, f32p, i64, f32p, f32p]
        L.pk_costmodel_adam_step.argtypes = [i32, f32p, f32p, f32p, f32p, i64, ctypes.c_float]
        L.pk_costmodel_params.argtypes = [vp, f32p, i32, ctypes.POINTER(ctypes.c_int)]
        L.pk_costmodel_save.argtypes = [vp, ctypes.c_char_p]
        L.pk_costmodel_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        L.pk_costmodel_free.argtypes = [vp]
        L.pk_costmodel_free.restype = None
        L.pk_costmodel_machine.argtypes = [vp]
        L.pk_costmodel_machine.restype = ctypes.c_char_p
        L.pk_case_table_set_costmodel.argtypes = [vp, vp]
        L.pk_costmodel_dtype.argtypes = [vp]
        L.pk_costmodel_set_dtype.argtypes = [vp, i32]
        L.pk_case_table_learned_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.pk_case_table_learned_measured.argtypes = [vp, ctypes.POINTER(i64)]
        L.pk_case_table_set_learned_margin.argtypes = [vp, ctypes.c_double]
        for name in ("pk_features", "pk_costmodel_train", "pk_costmodel_predict", "pk_costmodel_grad",
                     "pk_costmodel_adam_step", "pk_costmodel_params", "pk_costmodel_save", "pk_costmodel_load",
                     "pk_case_table_set_costmodel", "pk_case_table_learned_stats", "pk_costmodel_dtype",
                     "pk_case_table_learned_measured", "pk_case_table_set_learned_margin",
                     "pk_costmodel_set_dtype"):
            getattr(L, name).restype = i32
        for name in ("pk_machine_query", "pk_co_solve", "pk_case_table_build", "pk_case_table_describe",
                     "pk_case_table_lookup", "pk_select", "pk_matmul", "pk_launch_shape", "pk_measure"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PK_OK:
        raise PkError(rc, lib().pk_last_error().decode(errors="replace"))
    return rc


def last_error() -> str:
    return lib().pk_last_error().decode(errors="replace")


def pk_version() -> str:
    return lib().pk_version().decode()


def pk_instance_names():
    L = lib()
    return [L.pk_instance_name(i).decode() for i in range(L.pk_instance_count())]


def pk_machine_query(device: int = 0) -> pk_machine:
    m = pk_machine()
    _check(lib().pk_machine_query(device, ctypes.byref(m)))
    return m


def _text_call(fn, *args):
    need = ctypes.c_size_t(0)
    rc = fn(*args, None, 0, ctypes.byref(need))
    if rc not in (PK_OK, PK_ERR_BUFFER_TOO_SMALL):
        _check(rc)
    buf = ctypes.create_string_buffer(need.value)
    _check(fn(*args, buf, need.value, ctypes.byref(need)))
    return buf.value.decode()


def pk_co_solve(spec: str) -> dict:
    """Algorithms 1 and 2 on a family given in the library's text format."""
    return json.loads(_text_call(lib().pk_co_solve, spec.encode()))


class Table:
    """Owner of a pk_table handle."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.pk_case_table_free(h)

    @property
    def _as_parameter_(self):
        return self.handle


def pk_case_table_build(device: int = 0, override: pk_machine | None = None) -> Table:
    h = ctypes.c_void_p()
    _check(lib().pk_case_table_build(device, ctypes.byref(override) if override is not None else None,
                                     ctypes.byref(h)))
    return Table(h)


def pk_case_table_describe(tbl: Table) -> dict:
    return json.loads(_text_call(lib().pk_case_table_describe, tbl.handle))


def pk_case_table_lookup(tbl: Table, dtype, p: pk_params):
    """(leaf, variant) at program parameters p, or raises PkError."""
    leaf, var = ctypes.c_int32(-1), ctypes.c_int32(-1)
    _check(lib().pk_case_table_lookup(tbl.handle, _dt(dtype), ctypes.byref(p), ctypes.byref(leaf),
                                      ctypes.byref(var)))
    return leaf.value, var.value


def _dt(dtype) -> int:
    return DTYPES[dtype] if isinstance(dtype, str) else int(dtype)


def pk_select(tbl: Table, dtype, M: int, N: int, K: int, policy: int = PK_POLICY_CASE,
              allow_fallback: bool = False) -> pk_params:
    out = pk_params()
    rc = lib().pk_select(tbl.handle, _dt(dtype), M, N, K, policy, ctypes.byref(out))
    if rc == PK_ERR_COST_MODEL and allow_fallback:
        return out
    _check(rc)
    return out


def pk_select_operands(tbl: Table, dtype, A, B, policy: int = PK_POLICY_CASE, allow_fallback: bool = False):
    """pk_select for these device operands (A: (M, K), B: (K, N)): MFMA
    candidates as they would run on them (element loads on unaligned rows)."""
    M, K = A.shape
    K2, N = B.shape
    if K2 != K:
        raise ValueError("shape mismatch: A %s, B %s" % (tuple(A.shape), tuple(B.shape)))
    (a, lda), (b, ldb) = _operands((A, _in_bytes(dtype), "A"), (B, _in_bytes(dtype), "B"))
    out = pk_params()
    rc = lib().pk_select_operands(tbl.handle, _dt(dtype), a, lda, b, ldb, M, N, K, policy, ctypes.byref(out))
    if rc == PK_ERR_COST_MODEL and allow_fallback:
        return out
    _check(rc)
    return out


def pk_measure(tbl: Table, dtype, M: int, N: int, K: int, A=None, B=None, C=None):
    """[(pk_params, seconds per launch)] for every feasible candidate, timed on
    the given device tensors (or on scratch operands when A is None)."""
    if A is not None:
        if tuple(A.shape) != (M, K) or tuple(B.shape) != (K, N) or tuple(C.shape) != (M, N):
            raise ValueError("operand shapes do not match M, N, K")
        (a, lda), (b, ldb), (c, ldc) = _operands((A, _in_bytes(dtype), "A"), (B, _in_bytes(dtype), "B"),
                                                 (C, 4, "C"))
    else:
        a = b = c = None
        lda = ldb = ldc = 0
    n = ctypes.c_int(0)
    rc = lib().pk_measure(tbl.handle, _dt(dtype), a, lda, b, ldb, c, ldc, M, N, K, None, None, 0, ctypes.byref(n))
    if rc not in (PK_OK, PK_ERR_BUFFER_TOO_SMALL):
        _check(rc)
    cap = n.value
    ps = (pk_params * cap)()
    secs = (ctypes.c_double * cap)()
    _check(lib().pk_measure(tbl.handle, _dt(dtype), a, lda, b, ldb, c, ldc, M, N, K, ps, secs, cap,
                            ctypes.byref(n)))
    return [(ps[i], secs[i]) for i in range(n.value)]


def pk_select_transpose(tbl: Table, dtype, M: int, N: int, policy: int = PK_POLICY_CASE) -> pk_params:
    out = pk_params()
    _check(lib().pk_select_transpose(tbl.handle, _dt(dtype), M, N, policy, ctypes.byref(out)))
    return out


def pk_transpose(tbl: Table, p, dtype, A, C, stream=None):
    """C = A^T on the device (4-byte elements); A: (M, N), C: (N, M)."""
    M, N = A.shape
    if tuple(C.shape) != (N, M):
        raise ValueError("C must be (N, M)")
    (a, lda), (c, ldc) = _operands((A, 4, "A"), (C, 4, "C"))
    _check(lib().pk_transpose(tbl.handle, ctypes.byref(p) if p is not None else None, _dt(dtype), a, lda,
                              c, ldc, M, N, _stream(stream)))


def pk_select_madd(tbl: Table, dtype, M: int, N: int, policy: int = PK_POLICY_CASE) -> pk_params:
    out = pk_params()
    _check(lib().pk_select_madd(tbl.handle, _dt(dtype), M, N, policy, ctypes.byref(out)))
    return out


def pk_madd(tbl: Table, p, dtype, A, B, C, stream=None):
    """C = A + B on the device (f32 or wrapping i32); A, B, C: (M, N)."""
    M, N = A.shape
    if tuple(B.shape) != (M, N) or tuple(C.shape) != (M, N):
        raise ValueError("A, B and C must have the same shape")
    (a, lda), (b, ldb), (c, ldc) = _operands((A, 4, "A"), (B, 4, "B"), (C, 4, "C"))
    _check(lib().pk_madd(tbl.handle, ctypes.byref(p) if p is not None else None, _dt(dtype), a, lda,
                         b, ldb, c, ldc, M, N, _stream(stream)))


def pk_select_jacobi1d(tbl: Table, dtype, N: int, policy: int = PK_POLICY_CASE, steps: int = 1) -> pk_params:
    out = pk_params()
    _check(lib().pk_select_jacobi1d(tbl.handle, _dt(dtype), N, steps, policy, ctypes.byref(out)))
    return out


def pk_jacobi1d(tbl: Table, p, dtype, a, steps: int, stream=None):
    """`steps` time steps in place on the device array a of 2N elements (two
    copies of the length-N vector), one launch per step."""
    if a.dim() != 1 or a.numel() % 2 or not a.is_contiguous():
        raise ValueError("a must be a contiguous 1-D array of even length")
    _check(lib().pk_jacobi1d(tbl.handle, ctypes.byref(p) if p is not None else None, _dt(dtype),
                             ctypes.c_void_p(a.data_ptr()), a.numel() // 2, steps, _stream(stream)))


def pk_select_polydiv(tbl: Table, N: int, M: int, policy: int = PK_POLICY_CASE) -> pk_params:
    out = pk_params()
    _check(lib().pk_select_polydiv(tbl.handle, N, M, policy, ctypes.byref(out)))
    return out


def pk_polydiv(tbl: Table, p, a, b, P: int, stream=None):
    """Divides, in place on the device, the polynomial a (N int32 words holding
    residues in [0, P)) by the monic polynomial x^M + b (b: its M low
    coefficients); a returns the remainder in a[:M], zeros above."""
    for t in (a, b):
        if t.dim() != 1 or not t.is_contiguous() or t.element_size() != 4:
            raise ValueError("a and b must be contiguous 1-D arrays of 32-bit words")
    _check(lib().pk_polydiv(tbl.handle, ctypes.byref(p) if p is not None else None, ctypes.c_void_p(a.data_ptr()),
                            a.numel(), ctypes.c_void_p(b.data_ptr()), b.numel(), P, _stream(stream)))


def pk_kernel_name(tbl: Table, p: pk_params, dtype) -> str:
    r = lib().pk_kernel_name(tbl.handle, ctypes.byref(p), _dt(dtype))
    if r is None:
        raise PkError(PK_ERR_INVALID_ARG, last_error())
    return r.decode()


def pk_probe_valu_rate(tbl: Table, dtype) -> float:
    """Measured vector-ALU multiply-add ceiling, operations per second."""
    out = ctypes.c_double()
    _check(lib().pk_probe_valu_rate(tbl.handle, _dt(dtype), ctypes.byref(out)))
    return out.value


def pk_estimate(tbl: Table, p: pk_params, dtype, M: int, N: int, K: int, wide: bool = True) -> float:
    """The CASE policy's analytic seconds for one launch of p on M x N x K."""
    out = ctypes.c_double()
    _check(lib().pk_estimate(tbl.handle, ctypes.byref(p), _dt(dtype), M, N, K, 1 if wide else 0, ctypes.byref(out)))
    return out.value


def pk_launch_shape(tbl: Table, p: pk_params, dtype, M: int, N: int, K: int):
    g, b, l = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().pk_launch_shape(tbl.handle, ctypes.byref(p), _dt(dtype), M, N, K, ctypes.byref(g),
                                 ctypes.byref(b), ctypes.byref(l)))
    return g.value, b.value, l.value


def _ptr_ld(t, esize=None, what="matrix", device=True):
    """Device pointer and leading dimension of a row-major 2-D device tensor.

    Raises ValueError unless the tensor is 2-D with unit column stride, its
    rows do not overlap (stride(0) >= columns when it has several rows, so an
    expand()ed operand or an aliased output is refused), its elements have
    `esize` bytes (when given) and it lives on the GPU.  The leading dimension
    passed on is the tensor's own row stride (for a single row, which is the
    only row read, at least its column count)."""
    if t.dim() != 2:
        raise ValueError("%s must be 2-D, got %d dimensions" % (what, t.dim()))
    rows, cols = int(t.shape[0]), int(t.shape[1])
    if cols > 1 and t.stride(1) != 1:
        raise ValueError("%s must have unit column stride (stride %s)" % (what, tuple(t.stride())))
    if rows > 1 and t.stride(0) < cols:
        raise ValueError("%s rows overlap: row stride %d < %d columns" % (what, t.stride(0), cols))
    if esize is not None and t.element_size() != esize:
        raise ValueError("%s has %d-byte elements, the dtype needs %d" % (what, t.element_size(), esize))
    if device and not t.is_cuda:
        raise ValueError("%s must be a GPU tensor (got device %s)" % (what, t.device))
    ld = t.stride(0) if rows > 1 else max(t.stride(0), cols)
    return ctypes.c_void_p(t.data_ptr()), ld


def _operands(*specs):
    """[(pointer, ld)] for (tensor, element bytes, name) triples: every
    layout is checked before any device, so a malformed operand is reported
    as such whatever the others are."""
    for t, es, what in specs:
        _ptr_ld(t, es, what, device=False)
    return [_ptr_ld(t, es, what) for t, es, what in specs]


def _in_bytes(dtype) -> int:
    """Bytes per element of the operands A and B of a product of this dtype."""
    return 2 if _dt(dtype) == PK_BF16 else 4


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def pk_matmul(tbl: Table, p, dtype, A, B, C, accumulate: bool = False, stream=None):
    """C = [C +] A @ B on the device.  A: (M, K), B: (K, N), C: (M, N) torch
    tensors; for bf16, A and B hold bfloat16 (or int16 bit patterns) and C is
    float32.  p: a pk_params, or None for the CASE choice."""
    M, K = A.shape
    K2, N = B.shape
    if K2 != K or tuple(C.shape) != (M, N):
        raise ValueError("shape mismatch: A %s, B %s, C %s" % (tuple(A.shape), tuple(B.shape), tuple(C.shape)))
    (a, lda), (b, ldb), (c, ldc) = _operands((A, _in_bytes(dtype), "A"), (B, _in_bytes(dtype), "B"), (C, 4, "C"))
    _check(lib().pk_matmul(tbl.handle, ctypes.byref(p) if p is not None else None, _dt(dtype),
                           a, lda, b, ldb, c, ldc, M, N, K, 1 if accumulate else 0, _stream(stream)))


# ---------------------------------------------------------------------- cost model
PK_NFEATURES = 13


def _fbuf(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def pk_features(tbl: Table, p: pk_params, dtype, M: int, N: int, K: int, wide: bool = True):
    """wide: the operands' rows are aligned for the MFMA programs' 16-byte
    loads (packed operands: K and N multiples of 4 in f32, of 8 and 2 in bf16)."""
    import numpy as np
    out = np.zeros(PK_NFEATURES, dtype=np.float32)
    _check(lib().pk_features(tbl.handle, ctypes.byref(p), _dt(dtype), M, N, K, 1 if wide else 0,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def packed_rows_wide(dtype, N: int, K: int) -> bool:
    """Whether packed operands (lda = K, ldb = N) from 16-byte aligned bases
    have rows aligned for the MFMA programs' wide loads."""
    if _dt(dtype) == PK_BF16:
        return K % 8 == 0 and N % 8 == 0
    return K % 4 == 0 and N % 4 == 0


class CostModel:
    """Owner of a pk_costmodel handle."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.pk_costmodel_free(h)

    def params(self):
        import numpy as np
        n = ctypes.c_int(0)
        _check(lib().pk_costmodel_params(self.handle, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.float32)
        _check(lib().pk_costmodel_params(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         n.value, ctypes.byref(n)))
        return out

    def machine(self) -> str:
        return lib().pk_costmodel_machine(self.handle).decode()

    def dtype(self) -> str:
        """The element type whose timings the model was trained on."""
        code = lib().pk_costmodel_dtype(self.handle)
        _check(min(code, 0))
        return {v: k for k, v in DTYPES.items()}[code]

    def set_dtype(self, dtype):
        _check(lib().pk_costmodel_set_dtype(self.handle, _dt(dtype)))

    def predict(self, X, device: int = 0):
        import numpy as np
        X, px = _fbuf(X)
        out = np.zeros(X.shape[0], dtype=np.float32)
        _check(lib().pk_costmodel_predict(self.handle, device, px, X.shape[0],
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def save(self, path: str):
        _check(lib().pk_costmodel_save(self.handle, path.encode()))


def pk_costmodel_train(tbl: Table, X, seconds, epochs: int = 2000, lr: float = 3e-3, seed: int = 0):
    """Trains on the device; returns (CostModel, final loss)."""
    X, px = _fbuf(X)
    s, ps = _fbuf(seconds)
    h = ctypes.c_void_p()
    loss = ctypes.c_float(0)
    _check(lib().pk_costmodel_train(tbl.handle, px, ps, X.shape[0], epochs, lr, seed, ctypes.byref(h),
                                    ctypes.byref(loss)))
    return CostModel(h), loss.value


def load_shipped_models(tbl: Table):
    """Gives the table every cost model shipped in data/ for its machine
    (costmodel_<dtype>_<arch>.txt); returns the element types loaded.  A
    model for another machine is skipped."""
    arch = pk_case_table_describe(tbl)["machine"]["arch"].split(":")[0]
    loaded = []
    for dt in DTYPES:
        path = os.path.join(_HERE, "data", "costmodel_%s_%s.txt" % (dt, arch))
        if not os.path.exists(path):
            continue
        try:
            cm = pk_costmodel_load(path)
            pk_case_table_set_costmodel(tbl, cm)
        except PkError:
            continue
        loaded.append(cm.dtype())
    return loaded


def pk_costmodel_load(path: str) -> CostModel:
    h = ctypes.c_void_p()
    _check(lib().pk_costmodel_load(path.encode(), ctypes.byref(h)))
    return CostModel(h)


def pk_costmodel_grad(params, X, t, device: int = 0):
    """(gradient, loss) of the raw network on the device."""
    import numpy as np
    P, pp = _fbuf(params)
    X, px = _fbuf(X)
    T, pt = _fbuf(t)
    g = np.zeros(P.shape[0], dtype=np.float32)
    loss = ctypes.c_float(0)
    _check(lib().pk_costmodel_grad(device, pp, px, pt, X.shape[0], g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   ctypes.byref(loss)))
    return g, loss.value


def pk_costmodel_adam_step(params, grad, m, v, step: int, lr: float, device: int = 0):
    """One device Adam step; returns new (params, m, v)."""
    P, pp = _fbuf(params)
    P = P.copy()
    pp = P.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    G, pg = _fbuf(grad)
    Mv, pm = _fbuf(m)
    Mv = Mv.copy()
    pm = Mv.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    V, pv = _fbuf(v)
    V = V.copy()
    pv = V.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    _check(lib().pk_costmodel_adam_step(device, pp, pg, pm, pv, step, lr))
    return P, Mv, V


def pk_case_table_set_costmodel(tbl: Table, cm):
    _check(lib().pk_case_table_set_costmodel(tbl.handle, cm.handle if cm is not None else None))


def pk_case_table_learned_stats(tbl: Table):
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().pk_case_table_learned_stats(tbl.handle, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def pk_case_table_learned_measured(tbl: Table) -> int:
    """Candidates timed by the LEARNED policy's fallbacks, in total."""
    n = ctypes.c_int64(0)
    _check(lib().pk_case_table_learned_measured(tbl.handle, ctypes.byref(n)))
    return n.value


def pk_case_table_set_learned_margin(tbl: Table, margin: float):
    """The LEARNED policy's measurement margin (default 0.05; 0: never measure)."""
    _check(lib().pk_case_table_set_learned_margin(tbl.handle, float(margin)))


# ---------------------------------------------------------------------- many products
def _grouped_arrays(As, Bs, Cs, dtype):
    G = len(As)
    if not (len(Bs) == len(Cs) == G):
        raise ValueError("As, Bs, Cs must have the same length")
    I64 = ctypes.c_int64 * G
    P = ctypes.c_void_p * G
    M, N, K, lda, ldb, ldc = I64(), I64(), I64(), I64(), I64(), I64()
    a, b, c = P(), P(), P()
    for g, (A, B, C) in enumerate(zip(As, Bs, Cs)):
        m, k = A.shape
        k2, n = B.shape
        if k2 != k or tuple(C.shape) != (m, n):
            raise ValueError("shape mismatch in product %d" % g)
        M[g], N[g], K[g] = m, n, k
        (pa, la), (pb, lb), (pc, lc) = _operands((A, _in_bytes(dtype), "A[%d]" % g),
                                                 (B, _in_bytes(dtype), "B[%d]" % g), (C, 4, "C[%d]" % g))
        a[g], b[g], c[g] = pa.value, pb.value, pc.value
        lda[g], ldb[g], ldc[g] = la, lb, lc
    return G, (M, N, K, a, lda, b, ldb, c, ldc)


def _grouped_sigs(L):
    vp, i64p, i32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int
    arrs = [i64p, i64p, i64p, ctypes.POINTER(vp), i64p, ctypes.POINTER(vp), i64p, ctypes.POINTER(vp), i64p]
    if getattr(L, "_grouped_sigs", False):
        return
    L.pk_grouped_plan_create.argtypes = [vp, i32, ctypes.c_int32] + arrs + [ctypes.POINTER(pk_params), i32, i32,
                                                                              ctypes.POINTER(vp)]
    L.pk_grouped_plan_run.argtypes = [vp, vp]
    L.pk_grouped_plan_capture.argtypes = [vp]
    L.pk_grouped_plan_replay.argtypes = [vp, vp]
    L.pk_grouped_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(pk_params), ctypes.c_int32]
    L.pk_grouped_plan_kernel.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p)]
    L.pk_grouped_plan_destroy.argtypes = [vp]
    L.pk_grouped_plan_destroy.restype = None
    L.pk_matmul_batched.argtypes = [vp, i32, ctypes.c_int32] + arrs + [ctypes.POINTER(pk_params), vp]
    L.pk_matmul_batched_noalloc.argtypes = [vp, i32, ctypes.c_int32] + arrs + [ctypes.POINTER(pk_params), vp]
    for n in ("pk_grouped_plan_create", "pk_grouped_plan_run", "pk_grouped_plan_capture", "pk_grouped_plan_replay",
              "pk_grouped_plan_info", "pk_grouped_plan_kernel", "pk_matmul_batched", "pk_matmul_batched_noalloc"):
        getattr(L, n).restype = i32
    L._grouped_sigs = True


class GroupedPlan:
    """Owner of a pk_grouped_plan handle (keeps the operand tensors alive)."""

    def __init__(self, handle, G, keep):
        self.handle, self.G, self._keep = handle, G, keep

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.pk_grouped_plan_destroy(h)

    def run(self, stream=None):
        _check(lib().pk_grouped_plan_run(self.handle, _stream(stream)))

    def capture(self):
        _check(lib().pk_grouped_plan_capture(self.handle))

    def replay(self, stream=None):
        _check(lib().pk_grouped_plan_replay(self.handle, _stream(stream)))

    def info(self):
        n, t = ctypes.c_int32(0), ctypes.c_int64(0)
        chosen = (pk_params * max(self.G, 1))()
        _check(lib().pk_grouped_plan_info(self.handle, ctypes.byref(n), ctypes.byref(t), chosen, self.G))
        return n.value, t.value, [chosen[i] for i in range(self.G)]

    def kernels(self):
        """Names of the plan's launches' kernels, in launch order."""
        n = self.info()[0]
        out = []
        for i in range(n):
            name = ctypes.c_char_p()
            _check(lib().pk_grouped_plan_kernel(self.handle, i, ctypes.byref(name)))
            out.append(name.value.decode())
        return out


def pk_grouped_plan_create(tbl: Table, dtype, As, Bs, Cs, params=None, policy: int = PK_POLICY_CASE,
                           accumulate: bool = False) -> GroupedPlan:
    L = lib()
    _grouped_sigs(L)
    G, arrs = _grouped_arrays(As, Bs, Cs, dtype)
    ps = None
    if params is not None:
        ps = (pk_params * G)(*params)
    h = ctypes.c_void_p()
    _check(L.pk_grouped_plan_create(tbl.handle, _dt(dtype), G, *arrs, ps, policy, 1 if accumulate else 0,
                                    ctypes.byref(h)))
    return GroupedPlan(h, G, (As, Bs, Cs, arrs))


def pk_matmul_batched(tbl: Table, dtype, As, Bs, Cs, params=None, stream=None):
    L = lib()
    _grouped_sigs(L)
    G, arrs = _grouped_arrays(As, Bs, Cs, dtype)
    ps = (pk_params * G)(*params) if params is not None else None
    _check(L.pk_matmul_batched(tbl.handle, _dt(dtype), G, *arrs, ps, _stream(stream)))


def pk_matmul_batched_noalloc(tbl: Table, dtype, As, Bs, Cs, params=None, stream=None):
    """pk_matmul_batched without allocation: the launch's descriptors go to
    the library's per-device workspace (4 MiB); returns after the work."""
    L = lib()
    _grouped_sigs(L)
    G, arrs = _grouped_arrays(As, Bs, Cs, dtype)
    ps = (pk_params * G)(*params) if params is not None else None
    _check(L.pk_matmul_batched_noalloc(tbl.handle, _dt(dtype), G, *arrs, ps, _stream(stream)))
