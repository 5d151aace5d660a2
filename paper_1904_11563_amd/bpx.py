"""Thin ctypes binding of libbpx (include/bpx.h): argument marshalling only.

Every step of the coded product runs in the library: code construction and
the peeling schedule in its host C++ core, encode / GEMM / peel in its HIP
kernels.  Device arguments are torch tensors (float32, CUDA/HIP, row-major
with unit column stride); the current torch stream is used unless a stream
is given.  There is no fallback: importing this module fails if libbpx.so
is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# torch bundles its own HIP runtime (same soname as ROCm's).  Loading torch
# first makes libbpx bind to that runtime, so the process has one HIP runtime
# and device pointers and streams from torch are valid in the library.
import torch  # noqa: F401,E402

_HERE = os.path.dirname(os.path.abspath(__file__))
# BPX_LIBRARY selects another build of the same library (the host-sanitizer
# build that the CPU tests run); the default is the in-tree libbpx.so.
LIB_PATH = os.environ.get("BPX_LIBRARY") or os.path.join(_HERE, "libbpx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1904_11563_amd.build`")

_lib = C.CDLL(LIB_PATH)

# status codes / enums (mirror include/bpx.h)
OK, E_INVALID, E_UNDECODABLE, E_NOMEM, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
CODE_ARRAY_SEARCH, CODE_TABLE1, CODE_TABLE3, CODE_MOJETTE, CODE_IDENTITY = 0, 1, 2, 3, 4
PREC_F32, PREC_BF16, PREC_BF16X3, PREC_FP8, PREC_FP8X2 = 0, 1, 2, 3, 4
MODE_ERASURE, MODE_STRAGGLER, MODE_FULL, MODE_MIN = 0, 1, 2, 3

PREC_NAMES = {"f32": PREC_F32, "bf16": PREC_BF16, "bf16x3": PREC_BF16X3,
              "fp8": PREC_FP8, "fp8x2": PREC_FP8X2}
MODE_NAMES = {"erasure": MODE_ERASURE, "straggler": MODE_STRAGGLER,
              "full": MODE_FULL, "min": MODE_MIN}

EXPORTS = [
    "bpx_code_build", "bpx_code_from_csr", "bpx_code_info", "bpx_code_csr", "bpx_code_free",
    "bpx_plan_create", "bpx_plan_create2d", "bpx_plan_grid", "bpx_plan_info",
    "bpx_plan_schedule", "bpx_plan_peel_program", "bpx_plan_workspace_bytes",
    "bpx_plan_workspace_layout",
    "bpx_plan_upload", "bpx_plan_free", "bpx_encode", "bpx_coded_gemm", "bpx_peel_decode",
    "bpx_coded_matmul", "bpx_coded_matmul_noalloc", "bpx_coded_matmul_grouped",
    "bpx_group_workspace_bytes",
    "bpx_group_create", "bpx_group_launch", "bpx_group_launch_phase", "bpx_group_free",
    "bpx_tile_count", "bpx_set_tile_order", "bpx_set_tile_table", "bpx_force_tile",
    "bpx_set_fused_peel", "bpx_plan_fused", "bpx_plan_fused_program", "bpx_last_error",
]


class CodeParams(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("k", C.c_int32), ("b", C.c_int32),
                ("sigma_max", C.c_int32), ("restarts", C.c_int32), ("iters", C.c_int32),
                ("mojette_qe", C.c_int32), ("seed", C.c_uint64), ("walk", C.c_int32),
                ("reserved", C.c_int32)]


_p = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_u16p = C.POINTER(C.c_uint16)

_sig = {
    "bpx_code_build": (C.c_int, [C.POINTER(CodeParams), C.POINTER(_p)]),
    "bpx_code_from_csr": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, _i32p, _i32p, _u16p,
                                    C.POINTER(_p)]),
    "bpx_code_info": (C.c_int, [_p] + [_i32p] * 6),
    "bpx_code_csr": (C.c_int, [_p, C.POINTER(_i32p), C.POINTER(_i32p), C.POINTER(_u16p)]),
    "bpx_code_free": (None, [_p]),
    "bpx_plan_create": (C.c_int, [_p, _i32p, C.c_int32, C.c_int32, C.c_int32, C.c_int64,
                                  C.c_int64, C.c_int64, C.c_int32, C.POINTER(_p)]),
    "bpx_plan_create2d": (C.c_int, [_p, _i32p, C.c_int32, C.c_int32, C.c_int32, C.c_int64,
                                    C.c_int64, C.c_int64, C.c_int32, C.POINTER(_p)]),
    "bpx_plan_grid": (C.c_int, [_p, _i32p, C.POINTER(C.c_int64)]),
    "bpx_plan_info": (C.c_int, [_p] + [_i32p] * 5 + [C.POINTER(C.c_int64)]),
    "bpx_plan_schedule": (C.c_int, [_p] + [C.POINTER(_i32p)] * 5 + [C.POINTER(_u16p),
                                                                    C.POINTER(_i32p)]),
    "bpx_plan_peel_program": (C.c_int, [_p, C.POINTER(_i32p), _i32p, _i32p, C.POINTER(_i32p),
                                        _i32p, _i32p]),
    "bpx_plan_workspace_bytes": (C.c_int, [_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "bpx_plan_workspace_layout": (C.c_int, [_p, C.POINTER(C.c_size_t), C.c_int32]),
    "bpx_plan_upload": (C.c_int, [_p]),
    "bpx_plan_free": (None, [_p]),
    "bpx_encode": (C.c_int, [_p, _p, C.c_int64, _p, _p]),
    "bpx_coded_gemm": (C.c_int, [_p, _p, C.c_int64, _p, C.c_int64, _p, C.c_int64, _p,
                                 C.c_size_t, _p]),
    "bpx_peel_decode": (C.c_int, [_p, _p, C.c_size_t, _p, C.c_int64, _p]),
    "bpx_coded_matmul": (C.c_int, [_p, _p, C.c_int64, _p, C.c_int64, _p, C.c_int64, _p,
                                   C.c_size_t, _p]),
    "bpx_coded_matmul_noalloc": (C.c_int, [_p, _p, C.c_int64, _p, C.c_int64, _p, C.c_int64,
                                           _p]),
    "bpx_coded_matmul_grouped": (C.c_int, [C.POINTER(_p), C.POINTER(_p), C.POINTER(_p),
                                           C.POINTER(_p), C.c_int32, _p, C.c_size_t, _p]),
    "bpx_group_workspace_bytes": (C.c_int, [C.POINTER(_p), C.c_int32, C.POINTER(C.c_size_t)]),
    "bpx_group_create": (C.c_int, [C.POINTER(_p), C.POINTER(_p), C.POINTER(_p), C.POINTER(_p),
                                   C.c_int32, _p, C.c_size_t, C.POINTER(_p)]),
    "bpx_group_launch": (C.c_int, [_p, _p]),
    "bpx_group_launch_phase": (C.c_int, [_p, C.c_int32, _p]),
    "bpx_group_free": (None, [_p]),
    "bpx_tile_count": (C.c_int32, [C.c_int32]),
    "bpx_set_tile_table": (C.c_int, [_i32p, C.c_int32]),
    "bpx_force_tile": (C.c_int, [C.c_int32]),
    "bpx_set_tile_order": (C.c_int, [C.c_int32]),
    "bpx_set_fused_peel": (C.c_int, [C.c_int32]),
    "bpx_plan_fused": (C.c_int, [_p, _i32p]),
    "bpx_plan_fused_program": (C.c_int, [_p, C.POINTER(_i32p), _i32p, C.POINTER(_i32p), _i32p,
                                         C.POINTER(_i32p), _i32p]),
    "bpx_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class BpxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"bpx status {status}: {msg}")
        self.status = status


def _check(st, allow=()):
    if st != OK and st not in allow:
        raise BpxError(st, _lib.bpx_last_error().decode())
    return st


def last_error() -> str:
    return _lib.bpx_last_error().decode()


# ------------------------------------------------------------------ codes --

class Code:
    """A library-owned code handle."""

    def __init__(self, handle):
        self._h = handle if isinstance(handle, _p) else _p(handle)

    @classmethod
    def build(cls, kind, n=0, k=0, b=0, sigma_max=0, restarts=1, iters=0, mojette_qe=0, seed=0,
              walk=0):
        prm = CodeParams(kind, n, k, b, sigma_max, restarts, iters, mojette_qe, seed, walk, 0)
        h = _p()
        _check(_lib.bpx_code_build(C.byref(prm), C.byref(h)))
        return cls(h)

    @classmethod
    def table1(cls):
        return cls.build(CODE_TABLE1)

    @classmethod
    def table3(cls):
        return cls.build(CODE_TABLE3)

    @classmethod
    def identity(cls, k, b):
        return cls.build(CODE_IDENTITY, n=k, k=k, b=b)

    @classmethod
    def mojette(cls, k, b, n, qe=0):
        return cls.build(CODE_MOJETTE, n=n, k=k, b=b, mojette_qe=qe)

    @classmethod
    def search(cls, n, k, b, sigma_max, seed, restarts, iters, walk=0):
        return cls.build(CODE_ARRAY_SEARCH, n=n, k=k, b=b, sigma_max=sigma_max,
                         restarts=restarts, iters=iters, seed=seed, walk=walk)

    @classmethod
    def from_columns(cls, n, k, b, columns):
        col_ptr = [0]
        sym_ptr = [0]
        data = []
        for col in columns:
            for sym in col:
                data.extend(sorted(sym))
                sym_ptr.append(len(data))
            col_ptr.append(len(sym_ptr) - 1)
        cp = np.asarray(col_ptr, dtype=np.int32)
        sp = np.asarray(sym_ptr, dtype=np.int32)
        sd = np.asarray(data if data else [0], dtype=np.uint16)
        h = _p()
        _check(_lib.bpx_code_from_csr(n, k, b, cp.ctypes.data_as(_i32p), sp.ctypes.data_as(_i32p),
                                      sd.ctypes.data_as(_u16p), C.byref(h)))
        return cls(h)

    def info(self):
        v = [C.c_int32() for _ in range(6)]
        _check(_lib.bpx_code_info(self._h, *[C.byref(x) for x in v]))
        keys = ("n", "k", "b", "n_sym", "nnz", "max_degree")
        return dict(zip(keys, (x.value for x in v)))

    def csr(self):
        inf = self.info()
        cp, sp, sd = _i32p(), _i32p(), _u16p()
        _check(_lib.bpx_code_csr(self._h, C.byref(cp), C.byref(sp), C.byref(sd)))
        col_ptr = np.ctypeslib.as_array(cp, shape=(inf["n"] + 1,)).copy()
        sym_ptr = np.ctypeslib.as_array(sp, shape=(inf["n_sym"] + 1,)).copy()
        nnz = inf["nnz"]
        sym_data = np.ctypeslib.as_array(sd, shape=(nnz,)).copy() if nnz else np.zeros(0, np.uint16)
        return col_ptr, sym_ptr, sym_data

    def columns(self):
        """Columns as lists of sorted id tuples (same shape as the oracle's)."""
        col_ptr, sym_ptr, sym_data = self.csr()
        out = []
        for j in range(len(col_ptr) - 1):
            out.append([tuple(int(x) for x in sym_data[sym_ptr[g]:sym_ptr[g + 1]])
                        for g in range(col_ptr[j], col_ptr[j + 1])])
        return out

    def __del__(self):
        try:
            if getattr(self, "_h", None) and self._h.value:
                _lib.bpx_code_free(self._h)
                self._h = _p()
        except Exception:        # interpreter shutdown
            pass


# ------------------------------------------------------------------ plans --

class Plan:
    """A library-owned plan handle (prefix, schedule, device tables)."""

    def __init__(self, code: Code, arrival, n_lost, mode, M, K, N, prec=PREC_F32,
                 two_d=False):
        arr = np.ascontiguousarray(arrival, dtype=np.int32)
        self.code = code
        h = _p()
        create = _lib.bpx_plan_create2d if two_d else _lib.bpx_plan_create
        st = create(code._h, arr.ctypes.data_as(_i32p), len(arr), n_lost, mode,
                    M, K, N, prec, C.byref(h))
        _check(st, allow=(E_UNDECODABLE,))
        self._h = h
        self.M, self.K, self.N, self.prec, self.mode = M, K, N, prec, mode

    def info(self):
        v = [C.c_int32() for _ in range(5)]
        mb = C.c_int64()
        _check(_lib.bpx_plan_info(self._h, *[C.byref(x) for x in v], C.byref(mb)))
        keys = ("decodable", "prefix_m", "n_computed", "depth_max", "n_unrecovered")
        d = dict(zip(keys, (x.value for x in v)))
        d["decodable"] = bool(d["decodable"])
        d["Mb"] = mb.value
        return d

    @property
    def decodable(self):
        return self.info()["decodable"]

    def grid(self):
        """(grid, Nb): 1 and N for row-block plans."""
        g = C.c_int32()
        nb = C.c_int64()
        _check(_lib.bpx_plan_grid(self._h, C.byref(g), C.byref(nb)))
        return g.value, nb.value

    def schedule(self):
        inf = self.info()
        kb = self.code.info()["k"] * self.code.info()["b"]
        ptrs = [_i32p() for _ in range(6)]
        sd = _u16p()
        _check(_lib.bpx_plan_schedule(self._h, C.byref(ptrs[0]), C.byref(ptrs[1]),
                                      C.byref(ptrs[2]), C.byref(ptrs[3]), C.byref(ptrs[4]),
                                      C.byref(sd), C.byref(ptrs[5])))

        def arr(p, n, ctype=np.int32):
            return np.ctypeslib.as_array(p, shape=(n,)).copy() if n else np.zeros(0, ctype)

        nc = inf["n_computed"]
        sub_ptr = arr(ptrs[4], kb + 1)
        return {
            "computed": arr(ptrs[0], nc),
            "dest": arr(ptrs[1], nc),
            "releaser": arr(ptrs[2], kb),
            "depth": arr(ptrs[3], kb),
            "sub_ptr": sub_ptr,
            "sub_data": arr(sd, int(sub_ptr[-1]), np.uint16),
            "unrecovered": arr(ptrs[5], inf["n_unrecovered"]),
        }

    PEEL_FIELDS = ("s", "src", "nsub", "sub_off", "f64", "slot", "write", "brow", "bcol")

    def peel_program(self):
        """The decode's step program: {"steps": int32 [n_steps, 9] in
        PEEL_FIELDS order, "subs": the subtrahends' LDS slots, "n_slots"}."""
        st, sb = _i32p(), _i32p()
        n, w, ns, nsl = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.bpx_plan_peel_program(self._h, C.byref(st), C.byref(n), C.byref(w),
                                          C.byref(sb), C.byref(ns), C.byref(nsl)))
        steps = (np.ctypeslib.as_array(st, shape=(n.value * w.value,)).copy().reshape(n.value, w.value)
                 if n.value else np.zeros((0, 9), np.int32))
        subs = np.ctypeslib.as_array(sb, shape=(ns.value,)).copy() if ns.value else np.zeros(0, np.int32)
        return {"steps": steps, "subs": subs, "n_slots": nsl.value}

    def fused(self):
        """Whether coded_matmul takes the fused form (one launch) for this plan."""
        v = C.c_int32()
        _check(_lib.bpx_plan_fused(self._h, C.byref(v)))
        return bool(v.value)

    def fused_program(self):
        """The fused form's peel program: {"steps": int32 [n, 9] (PEEL_FIELDS,
        src = Y tile), "subs", "ytile" (per computed symbol), "n_ytiles"}."""
        st, sb, yt = _i32p(), _i32p(), _i32p()
        n, ns, ny = C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.bpx_plan_fused_program(self._h, C.byref(st), C.byref(n), C.byref(sb),
                                           C.byref(ns), C.byref(yt), C.byref(ny)))
        nc = self.info()["n_computed"]
        steps = (np.ctypeslib.as_array(st, shape=(n.value * 9,)).copy().reshape(n.value, 9)
                 if n.value else np.zeros((0, 9), np.int32))
        subs = np.ctypeslib.as_array(sb, shape=(ns.value,)).copy() if ns.value else np.zeros(0, np.int32)
        ytile = np.ctypeslib.as_array(yt, shape=(nc,)).copy() if nc and n.value else np.zeros(0, np.int32)
        return {"steps": steps, "subs": subs, "ytile": ytile, "n_ytiles": ny.value}

    def workspace_bytes(self):
        ws, enc = C.c_size_t(), C.c_size_t()
        _check(_lib.bpx_plan_workspace_bytes(self._h, C.byref(ws), C.byref(enc)))
        return ws.value, enc.value

    def workspace_layout(self):
        """Byte offsets of the workspace parts (see bpx_plan_workspace_layout)."""
        off = (C.c_size_t * 7)()
        _check(_lib.bpx_plan_workspace_layout(self._h, off, 7))
        return list(off)

    def upload(self):
        _check(_lib.bpx_plan_upload(self._h))

    def __del__(self):
        try:
            if getattr(self, "_h", None) and self._h.value:
                _lib.bpx_plan_free(self._h)
                self._h = _p()
        except Exception:        # interpreter shutdown
            pass


# ----------------------------------------------------------------- device --

def _mat(t, name, shape=None):
    """Pointer and leading dimension of a row-major float32 device matrix;
    shape, when given, is the (rows, cols) the plan expects."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or \
            t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D float32 device tensor with unit column stride")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, the plan expects {tuple(shape)}")
    return _p(t.data_ptr()), t.stride(0)


def _dense(t, name, shape):
    """Pointer of a dense (contiguous) row-major float32 device matrix of the
    given shape: grouped products bake lda = K, ldb = ldc = N."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or \
            not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous float32 device tensor of shape "
                         f"{tuple(shape)}")
    return _p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _p(s.cuda_stream)


def _ws(ws):
    import torch
    if ws is None:
        return _p(0), 0
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    return _p(ws.data_ptr()), ws.numel() * ws.element_size()


def alloc_workspace(plan: Plan, device="cuda"):
    import torch
    nbytes, _ = plan.workspace_bytes()
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def encode(plan: Plan, A, out, stream=None):
    import torch
    a, lda = _mat(A, "A", (plan.M, plan.K))
    _, need = plan.workspace_bytes()
    if not isinstance(out, torch.Tensor) or out.dtype != torch.float32 or not out.is_cuda or \
            not out.is_contiguous() or out.numel() * 4 < need:
        raise ValueError(f"out must be a contiguous float32 device tensor of at least "
                         f"{need} bytes")
    _check(_lib.bpx_encode(plan._h, a, lda, _p(out.data_ptr()), _stream(stream)))


def coded_gemm(plan: Plan, A, B, C_out, ws, stream=None):
    a, lda = _mat(A, "A", (plan.M, plan.K))
    b, ldb = _mat(B, "B", (plan.K, plan.N))
    c, ldc = _mat(C_out, "C", (plan.M, plan.N))
    w, wb = _ws(ws)
    _check(_lib.bpx_coded_gemm(plan._h, a, lda, b, ldb, c, ldc, w, wb, _stream(stream)))


def peel_decode(plan: Plan, ws, C_out, stream=None):
    c, ldc = _mat(C_out, "C", (plan.M, plan.N))
    w, wb = _ws(ws)
    _check(_lib.bpx_peel_decode(plan._h, w, wb, c, ldc, _stream(stream)))


def coded_matmul(plan: Plan, A, B, C_out, ws, stream=None):
    a, lda = _mat(A, "A", (plan.M, plan.K))
    b, ldb = _mat(B, "B", (plan.K, plan.N))
    c, ldc = _mat(C_out, "C", (plan.M, plan.N))
    w, wb = _ws(ws)
    _check(_lib.bpx_coded_matmul(plan._h, a, lda, b, ldb, c, ldc, w, wb, _stream(stream)))


def coded_matmul_noalloc(plan: Plan, A, B, C_out, stream=None):
    """bpx_coded_matmul with the library's static scratch array as workspace
    (the plan must have been uploaded; 32 MiB limit)."""
    a, lda = _mat(A, "A", (plan.M, plan.K))
    b, ldb = _mat(B, "B", (plan.K, plan.N))
    c, ldc = _mat(C_out, "C", (plan.M, plan.N))
    _check(_lib.bpx_coded_matmul_noalloc(plan._h, a, lda, b, ldb, c, ldc, _stream(stream)))


def _group_operands(plans, As, Bs, Cs):
    n = len(plans)
    if not (len(As) == len(Bs) == len(Cs) == n) or n < 1:
        raise ValueError("plans, A, B and C must be non-empty lists of one length")
    P = (_p * n)(*[p._h for p in plans])
    A = (_p * n)(*[_dense(a, f"A[{i}]", (p.M, p.K)) for i, (p, a) in enumerate(zip(plans, As))])
    B = (_p * n)(*[_dense(b, f"B[{i}]", (p.K, p.N)) for i, (p, b) in enumerate(zip(plans, Bs))])
    Cc = (_p * n)(*[_dense(c, f"C[{i}]", (p.M, p.N)) for i, (p, c) in enumerate(zip(plans, Cs))])
    return n, P, A, B, Cc


def coded_matmul_grouped(plans, As, Bs, Cs, ws, stream=None):
    n, P, A, B, Cc = _group_operands(plans, As, Bs, Cs)
    w, wb = _ws(ws)
    _check(_lib.bpx_coded_matmul_grouped(P, A, B, Cc, n, w, wb, _stream(stream)))


def group_workspace_bytes(plans):
    n = len(plans)
    P = (_p * n)(*[p._h for p in plans])
    b = C.c_size_t()
    _check(_lib.bpx_group_workspace_bytes(P, n, C.byref(b)))
    return b.value


class Group:
    """A grouped launch over many plans (bpx_group_*): operands and workspace
    are fixed at creation, so launch() can be captured in a HIP graph."""

    def __init__(self, plans, As, Bs, Cs, ws):
        n, P, A, B, Cc = _group_operands(plans, As, Bs, Cs)
        w, wb = _ws(ws)
        h = _p()
        _check(_lib.bpx_group_create(P, A, B, Cc, n, w, wb, C.byref(h)))
        self._h = h
        self._keep = (plans, As, Bs, Cs, ws)   # operands must outlive the group

    def launch(self, stream=None):
        _check(_lib.bpx_group_launch(self._h, _stream(stream)))

    def launch_phase(self, phase, stream=None):
        _check(_lib.bpx_group_launch_phase(self._h, phase, _stream(stream)))

    def __del__(self):
        try:
            if getattr(self, "_h", None) and self._h.value:
                _lib.bpx_group_free(self._h)
                self._h = _p()
        except Exception:        # interpreter shutdown
            pass


def tile_count(prec=PREC_F32):
    return _lib.bpx_tile_count(prec)


def set_tile_table(table):
    if table is None:
        _check(_lib.bpx_set_tile_table(None, 0))
        return
    t = np.ascontiguousarray(table, dtype=np.int32)
    _check(_lib.bpx_set_tile_table(t.ctypes.data_as(_i32p), len(t)))


def set_tile_order(group_m):
    _check(_lib.bpx_set_tile_order(group_m))


def force_tile(t):
    _check(_lib.bpx_force_tile(t))


def set_fused_peel(mode):
    """0: never fuse the peel into the GEMM; 1: small products (default);
    2: whenever the fused form fits."""
    _check(_lib.bpx_set_fused_peel(mode))
