"""Python binding of librlu: the MI355X sparse-projection randomized LU.

Argument marshalling only.  Every step of the decomposition runs in the HIP
library (``csrc/``, built into ``librlu.so``); torch provides device memory
(tensors' ``data_ptr()``) and the current HIP stream.  There is no CPU
fallback: without the built library every call raises.

Method: Aizenbud, Shabat & Averbuch, "Randomized LU decomposition using
sparse projections" (arXiv 1601.04280), Algorithm 1, with the exact
least-squares product of Corollary 3.2.  See ``include/rlu.h`` for the
conventions (pivot ties, zero pivots, parameter generator, real transform).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass
from typing import Optional

__all__ = [
    "RluError", "Context", "Factorization", "Server", "alloc_factors", "alloc_info", "info_dict", "workspace_size",
    "sketch_params", "sketch", "factor", "tall_lu",
    "library_path", "load_library", "PRECISIONS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "librlu.so")

RLU_OK, RLU_ERR_INVALID_ARG, RLU_ERR_NO_MEMORY, RLU_ERR_DEVICE, RLU_ERR_NUMERIC, RLU_ERR_AGAIN, \
    RLU_ERR_UNKNOWN_TICKET = range(7)
STATUS_NAMES = {0: "RLU_OK", 1: "RLU_ERR_INVALID_ARG", 2: "RLU_ERR_NO_MEMORY", 3: "RLU_ERR_DEVICE",
                4: "RLU_ERR_NUMERIC", 5: "RLU_ERR_AGAIN", 6: "RLU_ERR_UNKNOWN_TICKET"}
RLU_DENSE_ROW_MAJOR, RLU_CSR = 0, 1
RLU_F64, RLU_F32 = 0, 1
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2}
RLU_FLAG_VALIDATE = 1
RLU_FLAG_TIMING = 2
RLU_FLAG_EXCLUSIVE = 4
RLU_FLAG_TIMING_CONTRACT = 8
RLU_FLAG_HADAMARD = 16
RLU_FLAG_DETERMINISTIC = 32
RLU_FLAG_TRUNCATE = 64
STAGES = ["params", "sketch", "lu_y", "contract", "gram", "chol", "solve", "lu_b", "assemble"]


class RluError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Matrix(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("layout", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("values", ctypes.c_void_p), ("ld", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("nnz", ctypes.c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("l", ctypes.c_int32), ("s", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("k2", ctypes.c_int32), ("l2", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("zero_pivots_y", ctypes.c_int32),
                ("zero_pivots_b", ctypes.c_int32), ("nonfinite", ctypes.c_int32),
                ("timeouts", ctypes.c_int32), ("bad_index", ctypes.c_int32),
                ("zero_pivots_sel", ctypes.c_int32), ("reserved", ctypes.c_int32), ("min_gap_y", ctypes.c_double),
                ("min_gap_b", ctypes.c_double)]


INFO_WORDS = ctypes.sizeof(Info) // 4   # rlu_info as int32 words (device tensor)


def info_dict(info) -> dict:
    """Decode a device rlu_info record (int32 tensor of INFO_WORDS words)."""
    v = info.cpu()
    ints = v[:8].tolist()
    gaps = v[8:12].contiguous().view(_torch().float64).tolist()
    return {"status": ints[0], "zero_pivots_y": ints[1], "zero_pivots_b": ints[2], "nonfinite": ints[3],
            "timeouts": ints[4], "bad_index": ints[5], "zero_pivots_sel": ints[6],
            "min_gap_y": gaps[0], "min_gap_b": gaps[1]}


def alloc_info(device) -> object:
    """Storage of one rlu_info record; the call that fills it clears it on its own stream."""
    return _torch().empty(INFO_WORDS, dtype=_torch().int32, device=device)


class Factors(ctypes.Structure):
    _fields_ = [("L", ctypes.c_void_p), ("ldl", ctypes.c_int64), ("U", ctypes.c_void_p),
                ("ldu", ctypes.c_int64), ("perm_r", ctypes.c_void_p), ("perm_c", ctypes.c_void_p),
                ("ipiv_r", ctypes.c_void_p), ("ipiv_c", ctypes.c_void_p), ("Y", ctypes.c_void_p),
                ("ldy", ctypes.c_int64), ("Uy", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("ysel", ctypes.c_void_p), ("info", ctypes.c_void_p)]


_lib = None


def load_library():
    """Load librlu.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise RuntimeError(f"{library_path} is missing: build it with __graft_entry__.build() "
                           "(python paper_1601_04280_amd/build.py)")
    lib = ctypes.CDLL(library_path)
    P, I64, I32, U64, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "rlu_create": (I32, [I32, ctypes.POINTER(P)]),
        "rlu_destroy": (I32, [P]),
        "rlu_workspace_size": (I32, [P, ctypes.POINTER(Matrix), ctypes.POINTER(Params), ctypes.POINTER(SZ)]),
        "rlu_sketch_params": (I32, [ctypes.POINTER(Params), I64, P, P, P, P, P]),
        "rlu_sketch": (I32, [P, ctypes.POINTER(Matrix), ctypes.POINTER(Params), P, I64, P, SZ, P]),
        "rlu_sketch_noalloc": (I32, [P, ctypes.POINTER(Matrix), ctypes.POINTER(Params), P, I64, P]),
        "rlu_factor": (I32, [P, ctypes.POINTER(Matrix), ctypes.POINTER(Params), ctypes.POINTER(Factors),
                              P, SZ, P]),
        "rlu_tall_lu": (I32, [P, P, I64, I64, I64, P, P, P, P, P, P, SZ, P]),
        "rlu_tall_lu_workspace_size": (I32, [P, I64, I64, ctypes.POINTER(SZ)]),
        "rlu_serve_start": (I32, [P, SZ, I32]),
        "rlu_submit": (I32, [P, ctypes.POINTER(Matrix), ctypes.POINTER(Params), ctypes.POINTER(Factors),
                              ctypes.POINTER(U64)]),
        "rlu_poll": (I32, [P, U64]),
        "rlu_serve_stop": (I32, [P]),
        "rlu_serve_stats": (I32, [P, ctypes.POINTER(U64)]),
        "rlu_stage_times": (I32, [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(I32)]),
        "rlu_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != RLU_OK:
        msg = load_library().rlu_last_error().decode(errors="replace")
        raise RluError(status, msg)


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


_open_contexts = weakref.WeakSet()


@atexit.register
def _close_open_contexts():
    # Interpreter exit: destroy every context (its serving loop, streams and
    # events) while the HIP runtime is still whole, rather than from __del__
    # during module teardown, after the runtime's own exit handlers.
    for c in list(_open_contexts):
        try:
            c.close()
        except Exception:
            pass
    _default_ctx.clear()


class Context:
    """One rlu_ctx on a device, plus a cached workspace tensor."""

    def __init__(self, device: int = 0):
        lib = load_library()
        self.device = device
        self._h = ctypes.c_void_p()
        _check(lib.rlu_create(device, ctypes.byref(self._h)))
        self._ws = None
        _open_contexts.add(self)

    @property
    def handle(self):
        return self._h

    def workspace(self, nbytes: int):
        torch = _torch()
        nbytes = max(256, int(nbytes))
        if self._ws is None or self._ws.numel() < nbytes + 256:
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
        base = self._ws.data_ptr()
        off = (-base) % 256
        return base + off, self._ws.numel() - off

    def stage_times(self):
        """{stage: total ms} over calls made with RLU_FLAG_TIMING (or RLU_FLAG_TIMING_CONTRACT: the
        contraction only) since the last read, and the call count."""
        ms = (ctypes.c_float * len(STAGES))()
        calls = ctypes.c_int(0)
        _check(load_library().rlu_stage_times(self._h, ms, ctypes.byref(calls)))
        return {name: float(ms[i]) for i, name in enumerate(STAGES)}, calls.value

    def close(self):
        if self._h:
            load_library().rlu_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def _params(k, l, s, seed, precision="f64", flags=0, k2=0, l2=0) -> Params:
    return Params(int(k), int(l), int(s), PRECISIONS[precision], int(seed) & ((1 << 64) - 1),
                  int(flags), int(k2), int(l2), 0)


def _dense_matrix(A) -> Matrix:
    torch = _torch()
    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D CUDA (HIP) tensor")
    if A.stride(1) != 1:
        raise ValueError("A must be row major (stride(1) == 1)")
    if A.dtype == torch.float64:
        dt = RLU_F64
    elif A.dtype == torch.float32:
        dt = RLU_F32
    else:
        raise ValueError("A must be float64 or float32")
    return Matrix(A.shape[0], A.shape[1], RLU_DENSE_ROW_MAJOR, dt, A.data_ptr(), A.stride(0), None, None, 0)


def _csr_matrix(row_ptr, col, val, m, n) -> Matrix:
    torch = _torch()
    for t, dt in ((row_ptr, torch.int32), (col, torch.int32), (val, torch.float64)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError("CSR arrays must be contiguous CUDA tensors (int32, int32, float64)")
    return Matrix(int(m), int(n), RLU_CSR, RLU_F64, val.data_ptr(), 0, row_ptr.data_ptr(),
                  col.data_ptr(), int(val.numel()))


def sketch_params(n: int, l: int, s: int, seed: int, device: int = 0):
    """Device-drawn (h, sgn, d, sel) exactly as the compute calls draw them."""
    torch = _torch()
    dev = f"cuda:{device}"
    h = torch.empty(n, dtype=torch.int32, device=dev)
    sgn = torch.empty(n, dtype=torch.int8, device=dev)
    d = torch.empty(s, dtype=torch.int8, device=dev)
    sel = torch.empty(l, dtype=torch.int32, device=dev)
    p = _params(1, l, s, seed)
    _check(load_library().rlu_sketch_params(ctypes.byref(p), n, h.data_ptr(), sgn.data_ptr(),
                                            d.data_ptr(), sel.data_ptr(), _stream(device)))
    return h, sgn, d, sel


def sketch(A=None, *, k: int, l: int, s: int, seed: int, csr=None, ctx: Context = None, Y=None, flags: int = 0):
    """Algorithm 1 steps 1-2: Y = A Omega_1^T on the device (m x l, float64).
    flags: RLU_FLAG_* (RLU_FLAG_HADAMARD for the Walsh-Hadamard transform)."""
    torch = _torch()
    ctx = ctx or default_context()
    mat = _dense_matrix(A) if csr is None else _csr_matrix(*csr)
    p = _params(k, l, s, seed, flags=flags)
    lib = load_library()
    nbytes = ctypes.c_size_t()
    _check(lib.rlu_workspace_size(ctx.handle, ctypes.byref(mat), ctypes.byref(p), ctypes.byref(nbytes)))
    ws, wsb = ctx.workspace(nbytes.value)
    if Y is None:
        Y = torch.empty(mat.m, l, dtype=torch.float64, device=f"cuda:{ctx.device}")
    _check(lib.rlu_sketch(ctx.handle, ctypes.byref(mat), ctypes.byref(p), Y.data_ptr(), Y.stride(0), ws,
                          wsb, _stream(ctx.device)))
    return Y


def sketch_noalloc(A=None, *, k: int, l: int, s: int, seed: int, csr=None, ctx: Context = None, Y=None,
                   flags: int = 0):
    """``sketch`` through rlu_sketch_noalloc: the library's fixed per-device
    scratch array instead of a workspace (no device allocation inside the
    call).  Y (m x l, float64) is allocated here unless the caller passes it."""
    torch = _torch()
    ctx = ctx or default_context()
    mat = _dense_matrix(A) if csr is None else _csr_matrix(*csr)
    p = _params(k, l, s, seed, flags=flags)
    if Y is None:
        Y = torch.empty(mat.m, l, dtype=torch.float64, device=f"cuda:{ctx.device}")
    _check(load_library().rlu_sketch_noalloc(ctx.handle, ctypes.byref(mat), ctypes.byref(p), Y.data_ptr(),
                                             Y.stride(0), _stream(ctx.device)))
    return Y


@dataclass
class Factorization:
    L: object
    U: object
    perm_r: object
    perm_c: object
    ipiv_r: object
    ipiv_c: object
    Y: object
    Uy: object
    B: object
    info: object          # device int32[INFO_WORDS] (rlu_info)
    ysel: object = None   # RLU_FLAG_TRUNCATE: the k columns of Y kept

    def info_dict(self):
        return info_dict(self.info)


def workspace_size(A=None, *, k: int, l: int, s: int, precision: str = "f64", csr=None, ctx: Context = None,
                   k2: int = 0, l2: int = 0) -> int:
    """Bytes of workspace one decomposition of this problem needs."""
    ctx = ctx or default_context()
    mat = _dense_matrix(A) if csr is None else _csr_matrix(*csr)
    p = _params(k, l, s, 0, precision, 0, k2, l2)
    nbytes = ctypes.c_size_t()
    _check(load_library().rlu_workspace_size(ctx.handle, ctypes.byref(mat), ctypes.byref(p), ctypes.byref(nbytes)))
    return nbytes.value


def alloc_factors(m: int, n: int, l: int, device: int = 0, keep_intermediates: bool = False,
                  rank: int = None) -> Factorization:
    """Output buffers of one decomposition on the device: factors of rank
    ``rank`` (k for RLU_FLAG_TRUNCATE; l by default) from an l-column sketch."""
    torch = _torch()
    dev = f"cuda:{device}"
    f64, i32 = torch.float64, torch.int32
    r = l if rank is None else rank
    return Factorization(
        L=torch.empty(m, r, dtype=f64, device=dev), U=torch.empty(r, n, dtype=f64, device=dev),
        perm_r=torch.empty(m, dtype=i32, device=dev), perm_c=torch.empty(n, dtype=i32, device=dev),
        ipiv_r=torch.empty(r, dtype=i32, device=dev), ipiv_c=torch.empty(r, dtype=i32, device=dev),
        Y=torch.empty(m, l, dtype=f64, device=dev) if keep_intermediates else None,
        Uy=torch.empty(r, r, dtype=f64, device=dev) if keep_intermediates else None,
        B=torch.empty(r, n, dtype=f64, device=dev) if keep_intermediates else None,
        info=alloc_info(dev),
        ysel=torch.empty(r, dtype=i32, device=dev) if rank is not None else None)


def _factors(out: Factorization) -> Factors:
    return Factors(out.L.data_ptr(), out.L.stride(0), out.U.data_ptr(), out.U.stride(0), out.perm_r.data_ptr(),
                   out.perm_c.data_ptr(), _ptr(out.ipiv_r), _ptr(out.ipiv_c), _ptr(out.Y),
                   out.Y.stride(0) if out.Y is not None else 0, _ptr(out.Uy), _ptr(out.B), _ptr(out.ysel),
                   out.info.data_ptr())


def factor(A=None, *, k: int, l: int, s: int, seed: int, precision: str = "f64", csr=None,
           ctx: Context = None, keep_intermediates: bool = False, check: bool = True, flags: int = 0,
           out: Factorization = None, k2: int = 0, l2: int = 0) -> Factorization:
    """PAQ ~ LU on the device.  ``check`` synchronises and raises on a device-side error.

    ``k2 > 0`` computes B through the second projection Omega_2 (k2 x m, SEM
    width ``l2``) of Algorithm 1 steps 4-5 instead of the exact product."""
    torch = _torch()
    ctx = ctx or default_context()
    mat = _dense_matrix(A) if csr is None else _csr_matrix(*csr)
    m, n = mat.m, mat.n
    p = _params(k, l, s, seed, precision, flags, k2, l2)
    lib = load_library()
    nbytes = ctypes.c_size_t()
    _check(lib.rlu_workspace_size(ctx.handle, ctypes.byref(mat), ctypes.byref(p), ctypes.byref(nbytes)))
    ws, wsb = ctx.workspace(nbytes.value)
    if out is None:
        out = alloc_factors(m, n, l, ctx.device, keep_intermediates,
                            rank=k if flags & RLU_FLAG_TRUNCATE else None)
    f = _factors(out)
    _check(lib.rlu_factor(ctx.handle, ctypes.byref(mat), ctypes.byref(p), ctypes.byref(f), ws, wsb,
                          _stream(ctx.device)))
    if check:
        st = int(out.info[0].item())
        if st != RLU_OK:
            raise RluError(st, f"device-side failure, info={out.info_dict()}")
    return out


class Server:
    """Continuous batching of independent decompositions on one device
    (rlu_serve_start / rlu_submit / rlu_poll / rlu_serve_stop).

    Inputs and outputs stay referenced here until their ticket retires.  The
    library runs requests on its own streams: inputs written by torch must be
    complete before submit (``sync_inputs`` synchronises the current stream).
    """

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 4, device: int = 0):
        self.ctx = Context(device)
        self._live = {}
        _check(load_library().rlu_serve_start(self.ctx.handle, int(hbm_budget_bytes), int(max_inflight)))
        self._running = True

    def submit(self, A=None, *, k: int, l: int, s: int, seed: int, precision: str = "f64", csr=None,
               out: Factorization = None, keep_intermediates: bool = False, sync_inputs: bool = True,
               k2: int = 0, l2: int = 0, flags: int = 0) -> int:
        torch = _torch()
        mat = _dense_matrix(A) if csr is None else _csr_matrix(*csr)
        p = _params(k, l, s, seed, precision, flags, k2, l2)
        if out is None:
            out = alloc_factors(mat.m, mat.n, l, self.ctx.device, keep_intermediates,
                                rank=k if flags & RLU_FLAG_TRUNCATE else None)
        if sync_inputs:
            torch.cuda.current_stream(self.ctx.device).synchronize()
        f = _factors(out)
        ticket = ctypes.c_uint64(0)
        _check(load_library().rlu_submit(self.ctx.handle, ctypes.byref(mat), ctypes.byref(p), ctypes.byref(f),
                                         ctypes.byref(ticket)))
        self._live[ticket.value] = (A, csr, out)
        return ticket.value

    def poll(self, ticket: int):
        """The Factorization once the request is complete, else None; raises on failure."""
        st = load_library().rlu_poll(self.ctx.handle, ctypes.c_uint64(ticket))
        if st == RLU_ERR_AGAIN:
            return None
        entry = self._live.pop(ticket, None)
        _check(st)
        return entry[2] if entry else None

    def wait(self, ticket: int, timeout_s: float = 120.0):
        import time
        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"ticket {ticket} not complete after {timeout_s} s")
            time.sleep(20e-6)

    def stats(self) -> dict:
        """Serving-loop counters (rlu_serve_stats)."""
        v = (ctypes.c_uint64 * 8)()
        _check(load_library().rlu_serve_stats(self.ctx.handle, v))
        return {"exclusive_slot": bool(v[0]), "cus": int(v[1]), "graph_launches": int(v[2]),
                "graph_updates": int(v[3]), "graph_builds": int(v[4]), "direct_fallbacks": int(v[5])}

    def stop(self):
        if self._running:
            _check(load_library().rlu_serve_stop(self.ctx.handle))
            self._running = False
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()
        self.ctx.close()


def tall_lu(X, ctx: Context = None, check: bool = True):
    """Row-pivoted LU of a tall float64 device matrix: returns (Lhat, U, perm, ipiv, info)."""
    torch = _torch()
    ctx = ctx or default_context()
    rows, cols = X.shape
    lib = load_library()
    nbytes = ctypes.c_size_t()
    _check(lib.rlu_tall_lu_workspace_size(ctx.handle, rows, cols, ctypes.byref(nbytes)))
    ws, wsb = ctx.workspace(nbytes.value)
    dev = X.device
    Lhat = torch.empty(rows, cols, dtype=torch.float64, device=dev)
    U = torch.empty(cols, cols, dtype=torch.float64, device=dev)
    perm = torch.empty(rows, dtype=torch.int32, device=dev)
    ipiv = torch.empty(cols, dtype=torch.int32, device=dev)
    info = alloc_info(dev)
    _check(lib.rlu_tall_lu(ctx.handle, X.data_ptr(), rows, cols, X.stride(0), Lhat.data_ptr(), U.data_ptr(),
                           perm.data_ptr(), ipiv.data_ptr(), info.data_ptr(), ws, wsb, _stream(ctx.device)))
    if check and int(info[0].item()) != RLU_OK:
        raise RluError(int(info[0].item()), f"device-side failure, info={info.tolist()}")
    return Lhat, U, perm, ipiv, info
