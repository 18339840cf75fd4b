"""Thin ctypes binding of libada (the C ABI in include/ada.h).

Argument marshalling only: tensors are checked, laid out column-major, given a
workspace from PyTorch's caching allocator and handed to ``ada_solve`` with the
current HIP stream. Every step of the solve runs in the library's kernels.
Importing this module does not load the library; the first call does, and it
raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libada.so")

OK, ERR_ARG, ERR_NONFINITE, ERR_SINGULAR, ERR_NOMEM, ERR_HIP, ERR_FALLBACK_INFEASIBLE = 0, -1, -2, -3, -4, -5, -6
PENDING = 1
CLASS_GENERAL, CLASS_BANDED, CLASS_TRI_UPPER, CLASS_TRI_LOWER, CLASS_SYMPD, CLASS_SYM = 0, 1, 2, 3, 4, 5
ROUTE_NONE, ROUTE_BAND_LU, ROUTE_TRI, ROUTE_CHOL, ROUTE_LU, ROUTE_SVD, ROUTE_LDLT = range(7)
# routes the paper names as future work (Section V), off by default: bits of Opts.extensions
EXT_SYM = 1
EXTENSIONS = {"sym": EXT_SYM}
LAYOUT_DENSE, LAYOUT_BAND = 0, 1
PREC_FP64, PREC_FP32_IR, PREC_BF16_IR = 0, 1, 2
PRECISIONS = {"fp64": PREC_FP64, "fp32_ir": PREC_FP32_IR, "bf16_ir": PREC_BF16_IR}
# kernel families of the instrumentation (ADA_KF_*)
KERNEL_FAMILIES = ("gemm", "panel", "laswp", "trsm_block", "potrf", "trsv", "gbtrf", "gbtrs", "detect", "jacobi")
CLASS_NAMES = {0: "general", 1: "banded", 2: "tri_upper", 3: "tri_lower", 4: "sympd", 5: "sym"}
ROUTE_NAMES = {0: "none", 1: "band_lu", 2: "tri", 3: "chol", 4: "lu", 5: "svd", 6: "ldlt"}


class Opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("no_approx", ctypes.c_int32),
                ("rcond_threshold", ctypes.c_double), ("layout", ctypes.c_int32),
                ("kl_in", ctypes.c_int32), ("ku_in", ctypes.c_int32), ("force_general", ctypes.c_int32),
                ("want_berr", ctypes.c_int32), ("precision", ctypes.c_int32), ("extensions", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("cls", ctypes.c_int32), ("kl", ctypes.c_int32), ("ku", ctypes.c_int32),
                ("route", ctypes.c_int32), ("chol_failed", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("info", ctypes.c_int32), ("rank", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("nsolves", ctypes.c_int32), ("refine_iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rcond", ctypes.c_double), ("berr", ctypes.c_double)]


class BatchedShape(ctypes.Structure):
    """ada_batched_shape: the launch shape of the batched solve (speed only, results identical)."""
    _fields_ = [("buckets", ctypes.c_int32), ("max_n", ctypes.c_int32 * 3), ("wg_per_cu", ctypes.c_int32 * 3),
                ("workgroups", ctypes.c_int32 * 3), ("stage_cols", ctypes.c_int32)]

    def as_dict(self):
        k = self.buckets
        return {"max_n": list(self.max_n[:k]), "wg_per_cu": list(self.wg_per_cu[:k]),
                "workgroups": list(self.workgroups[:k]), "stage_cols": self.stage_cols}


def batched_shape(max_n=(256,), wg_per_cu=None, workgroups=None, stage_cols=8) -> BatchedShape:
    """An ada_batched_shape: one entry per range of orders (largest first)."""
    k = len(max_n)
    wpc = list(wg_per_cu or [1] * k)
    wg = list(workgroups or [256 * w for w in wpc])
    s = BatchedShape()
    s.buckets = k
    for j in range(k):
        s.max_n[j], s.wg_per_cu[j], s.workgroups[j] = int(max_n[j]), int(wpc[j]), int(wg[j])
    s.stage_cols = int(stage_cols)
    return s


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nrhs", ctypes.c_int32), ("lda", ctypes.c_int32), ("ldb", ctypes.c_int32),
                ("ldx", ctypes.c_int32), ("pad", ctypes.c_int32), ("a_off", ctypes.c_int64),
                ("b_off", ctypes.c_int64), ("x_off", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nrhs", ctypes.c_int32), ("lda", ctypes.c_int32), ("ldb", ctypes.c_int32),
                ("ldx", ctypes.c_int32), ("keep_factor", ctypes.c_int32), ("A", ctypes.c_void_p),
                ("reuse", ctypes.c_uint64), ("B", ctypes.c_void_p), ("X", ctypes.c_void_p), ("opts", Opts)]


class AdaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ada error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libada.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        L.ada_create.argtypes = [ctypes.POINTER(vp), i]
        L.ada_create.restype = i
        L.ada_destroy.argtypes = [vp]
        L.ada_destroy.restype = None
        L.ada_last_error.argtypes = []
        L.ada_last_error.restype = ctypes.c_char_p
        L.ada_opts_default.argtypes = [ctypes.POINTER(Opts)]
        L.ada_opts_default.restype = None
        L.ada_workspace_size.argtypes = [i, i, ctypes.POINTER(Opts)]
        L.ada_workspace_size.restype = sz
        L.ada_solve.argtypes = [vp, i, i, vp, i, vp, i, vp, i, vp, sz, ctypes.POINTER(Opts), ctypes.POINTER(Result), vp]
        L.ada_solve.restype = i
        L.ada_solve_noalloc.argtypes = [vp, i, i, vp, i, vp, i, vp, i, ctypes.POINTER(Opts), ctypes.POINTER(Result),
                                        vp]
        L.ada_solve_noalloc.restype = i
        L.ada_batched_workspace_size.argtypes = [i]
        L.ada_batched_workspace_size.restype = sz
        L.ada_solve_batched.argtypes = [vp, i, vp, vp, vp, vp, vp, sz, ctypes.POINTER(Opts), vp, vp]
        L.ada_solve_batched.restype = i
        bsp = ctypes.POINTER(BatchedShape)
        L.ada_set_batched_shape.argtypes = [vp, i, bsp]
        L.ada_set_batched_shape.restype = i
        L.ada_get_batched_shape.argtypes = [vp, i, bsp]
        L.ada_get_batched_shape.restype = i
        L.ada_autotune_batched.argtypes = [vp, i, vp, vp, vp, vp, vp, sz, ctypes.POINTER(Opts), vp, vp, bsp,
                                           ctypes.POINTER(ctypes.c_double)]
        L.ada_autotune_batched.restype = i
        L.ada_profile_enable.argtypes = [vp, i]
        L.ada_profile_enable.restype = i
        L.ada_profile_families.argtypes = [vp, ctypes.c_uint]
        L.ada_profile_families.restype = i
        L.ada_profile_reset.argtypes = [vp]
        L.ada_profile_reset.restype = i
        L.ada_autotune_band.argtypes = [vp, i, i, i, i, vp, ctypes.POINTER(i), ctypes.POINTER(ctypes.c_double)]
        L.ada_autotune_band.restype = i
        L.ada_profile_read.argtypes = [vp, i, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.ada_profile_read.restype = i
        u64, dp = ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)
        L.ada_server_create.argtypes = [vp, vp, sz, i, ctypes.POINTER(vp)]
        L.ada_server_create.restype = i
        L.ada_server_destroy.argtypes = [vp]
        L.ada_server_destroy.restype = None
        L.ada_request_footprint.argtypes = [ctypes.POINTER(Request)]
        L.ada_request_footprint.restype = sz
        L.ada_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(u64)]
        L.ada_submit.restype = i
        L.ada_poll.argtypes = [vp, u64, ctypes.POINTER(Result), ctypes.POINTER(u64), ctypes.c_int64]
        L.ada_poll.restype = i
        L.ada_poll_timed.argtypes = [vp, u64, ctypes.POINTER(Result), ctypes.POINTER(u64), ctypes.c_int64, dp, dp]
        L.ada_poll_timed.restype = i
        L.ada_factor_release.argtypes = [vp, u64]
        L.ada_factor_release.restype = i
        L.ada_server_usage.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(i), ctypes.POINTER(i)]
        L.ada_server_usage.restype = i
        _lib = L
    return _lib


def last_error() -> str:
    return lib().ada_last_error().decode(errors="replace")


def make_opts(no_approx=False, rcond_threshold=-1.0, layout=LAYOUT_DENSE, kl_in=0, ku_in=0, force_general=False,
              want_berr=True, precision="fp64", extensions=()) -> Opts:
    o = Opts()
    lib().ada_opts_default(ctypes.byref(o))
    o.no_approx = int(no_approx)
    o.rcond_threshold = float(rcond_threshold)
    o.layout = int(layout)
    o.kl_in = int(kl_in)
    o.ku_in = int(ku_in)
    o.force_general = int(force_general)
    o.want_berr = int(want_berr)
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
    o.precision = PRECISIONS[precision]
    bits = 0
    for e in extensions:
        if e not in EXTENSIONS:
            raise ValueError(f"extensions must be among {sorted(EXTENSIONS)}")
        bits |= EXTENSIONS[e]
    o.extensions = bits
    return o


def workspace_size(n: int, nrhs: int, opts: Opts | None = None) -> int:
    return int(lib().ada_workspace_size(n, nrhs, ctypes.byref(opts) if opts is not None else None))


class Context:
    """Owns an ada_ctx bound to one HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        rc = lib().ada_create(ctypes.byref(h), int(device))
        if rc != OK:
            raise AdaError(rc, last_error())
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().ada_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, on: bool = True, families=None):
        """Time kernel launches of the given families (names of KERNEL_FAMILIES; None: all)."""
        mask = 0xFFFFFFFF if families is None else sum(1 << KERNEL_FAMILIES.index(f) for f in families)
        lib().ada_profile_families(self.handle, mask)
        lib().ada_profile_enable(self.handle, int(on))

    def profile_reset(self):
        lib().ada_profile_reset(self.handle)

    def autotune_band(self, n: int, kl: int, ku: int, nrhs: int = 1):
        """Time the band solve's LDS staging pieces for this order and these widths on a synthetic
        factor and keep the fastest in this context. Returns (piece, ms per solve)."""
        import torch
        st = torch.cuda.current_stream(self.device).cuda_stream
        piece, ms = ctypes.c_int(), ctypes.c_double()
        rc = lib().ada_autotune_band(self.handle, int(n), int(kl), int(ku), int(nrhs), ctypes.c_void_p(st),
                                     ctypes.byref(piece), ctypes.byref(ms))
        if rc != OK:
            raise AdaError(rc, last_error())
        return piece.value, ms.value

    def profile_read(self, family: str):
        """(launches, total_ms, algorithmic flops, algorithmic bytes) of one kernel family."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        fl = ctypes.c_double()
        by = ctypes.c_double()
        rc = lib().ada_profile_read(self.handle, KERNEL_FAMILIES.index(family), ctypes.byref(n), ctypes.byref(ms),
                                    ctypes.byref(fl), ctypes.byref(by))
        if rc != OK:
            raise AdaError(rc, last_error())
        return n.value, ms.value, fl.value, by.value

    def profile_all(self) -> dict:
        return {f: self.profile_read(f) for f in KERNEL_FAMILIES}


_contexts: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    c = _contexts.get(device)
    if c is None:
        c = Context(device)
        _contexts[device] = c
    return c


def _colmajor(t):
    """A column-major view of a 2-D tensor (copies only when needed)."""
    import torch
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    if t.dtype != torch.float64:
        raise TypeError("ada works on float64 tensors")
    if t.shape[1] == 1:
        return t if t.stride(0) == 1 else t.contiguous()
    if t.stride(0) == 1 and t.stride(1) >= max(1, t.shape[0]):
        return t
    return t.t().contiguous().t()


def _ld(t) -> int:
    """Leading dimension of a column-major 2-D tensor (a single column has ld = rows)."""
    return t.stride(1) if t.shape[1] > 1 else max(1, t.shape[0])


@dataclass
class SolveResult:
    cls: str
    kl: int
    ku: int
    route: str
    chol_failed: bool
    fallback: int
    info: int
    rank: int
    sweeps: int
    nsolves: int
    rcond: float
    berr: float
    status: int = OK
    refine_iters: int = 0


def _result(r: Result, status: int) -> SolveResult:
    return SolveResult(CLASS_NAMES.get(r.cls, str(r.cls)), r.kl, r.ku, ROUTE_NAMES.get(r.route, str(r.route)),
                       bool(r.chol_failed), r.fallback, r.info, r.rank, r.sweeps, r.nsolves, r.rcond, r.berr, status,
                       r.refine_iters)


def solve(A, B, *, no_approx=False, rcond_threshold=-1.0, force_general=False, want_berr=True, layout="dense",
          kl_in=0, ku_in=0, out=None, work=None, ctx: Context | None = None, raise_on_error=True, precision="fp64",
          extensions=()):
    """Adaptive solve of A X = B on the GPU.

    extensions: "sym" (plain symmetric matrices by Bunch-Kaufman LDL^T), the route the paper names
    as future work.

    A: (n, n) float64 CUDA tensor, or for layout="band" the (kl_in+ku_in+1, n)
    LAPACK band storage (A[ku_in+i-j, j] = A(i, j)). B: (n,) or (n, nrhs).
    Returns (X, SolveResult). On ERR_SINGULAR (no_approx) X holds the routed
    solution and the result says why the fallback was due.
    """
    import torch
    dev = A.device
    if dev.type != "cuda":
        raise ValueError("A must be a CUDA tensor")
    vec = B.dim() == 1
    Ac = _colmajor(A)
    Bc = _colmajor(B)
    n = Bc.shape[0]
    nrhs = Bc.shape[1]
    lay = LAYOUT_BAND if layout == "band" else LAYOUT_DENSE
    if lay == LAYOUT_DENSE and (Ac.shape[0] != Ac.shape[1] or Ac.shape[0] != n):
        raise ValueError("A must be n x n and match B")
    if lay == LAYOUT_BAND and Ac.shape[1] != n:
        raise ValueError("band storage must have n columns")
    opts = make_opts(no_approx, rcond_threshold, lay, kl_in, ku_in, force_general, want_berr, precision, extensions)
    ws = workspace_size(n, nrhs, opts)
    if ws == 0:
        raise ValueError("invalid shape for the workspace query")
    if work is None or work.numel() < ws:
        work = torch.empty(ws, dtype=torch.uint8, device=dev)
    if out is None:
        X = torch.empty((nrhs, n), dtype=torch.float64, device=dev).t()
    else:
        X = out
    c = ctx or context(dev.index or 0)
    res = Result()
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = lib().ada_solve(c.handle, n, nrhs, Ac.data_ptr(), _ld(Ac), Bc.data_ptr(), _ld(Bc),
                         X.data_ptr(), _ld(X), work.data_ptr(), work.numel(), ctypes.byref(opts),
                         ctypes.byref(res), ctypes.c_void_p(stream))
    if rc not in (OK, ERR_SINGULAR):
        if raise_on_error:
            raise AdaError(rc, last_error())
        return None, SolveResult("", -1, -1, "none", False, 0, 0, 0, 0, 0, math.nan, math.nan, rc)
    out_x = X[:, 0] if vec else X
    return out_x, _result(res, rc)


NOALLOC_SCRATCH_BYTES = 256 << 20  # ADA_NOALLOC_SCRATCH_BYTES


def solve_noalloc(A, B, *, out=None, ctx: Context | None = None, raise_on_error=True, **opt_kw):
    """ada_solve_noalloc: the solve of `solve` with the library's fixed per-GPU scratch as its
    workspace (nothing is allocated; X must be given or is allocated here, before the call).
    Same options as `solve` (no_approx, rcond_threshold, force_general, want_berr, layout, kl_in,
    ku_in, precision, extensions)."""
    import torch
    dev = A.device
    if dev.type != "cuda":
        raise ValueError("A must be a CUDA tensor")
    vec = B.dim() == 1
    Ac = _colmajor(A)
    Bc = _colmajor(B)
    n, nrhs = Bc.shape[0], Bc.shape[1]
    lay = LAYOUT_BAND if opt_kw.pop("layout", "dense") == "band" else LAYOUT_DENSE
    opts = make_opts(layout=lay, **opt_kw)
    X = out if out is not None else torch.empty((nrhs, n), dtype=torch.float64, device=dev).t()
    c = ctx or context(dev.index or 0)
    res = Result()
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = lib().ada_solve_noalloc(c.handle, n, nrhs, Ac.data_ptr(), _ld(Ac), Bc.data_ptr(), _ld(Bc), X.data_ptr(),
                                 _ld(X), ctypes.byref(opts), ctypes.byref(res), ctypes.c_void_p(stream))
    if rc not in (OK, ERR_SINGULAR):
        if raise_on_error:
            raise AdaError(rc, last_error())
        return None, SolveResult("", -1, -1, "none", False, 0, 0, 0, 0, 0, math.nan, math.nan, rc)
    return (X[:, 0] if vec else X), _result(res, rc)


class Batch:
    """Many independent small systems packed once into device pools (column-major,
    one descriptor each), solved by one ada_solve_batched launch per run()."""

    def __init__(self, As, Bs, device="cuda:0", no_approx=False, rcond_threshold=-1.0, force_general=False,
                 want_berr=True, precision="fp64", ctx: Context | None = None, extensions=()):
        import numpy as np
        import torch
        if len(As) != len(Bs) or not As:
            raise ValueError("As and Bs must be non-empty lists of equal length")
        self.count = len(As)
        dev = torch.device(device)
        descs = (Desc * self.count)()
        a_parts, b_parts = [], []
        ao = bo = xo = 0
        self.shapes = []
        for k, (a, b) in enumerate(zip(As, Bs)):
            a = np.asarray(a, dtype=np.float64)
            b = np.asarray(b, dtype=np.float64)
            if b.ndim == 1:
                b = b[:, None]
            n, nr = a.shape[0], b.shape[1]
            descs[k] = Desc(n, nr, n, n, n, 0, ao, bo, xo)
            a_parts.append(np.asfortranarray(a).ravel(order="F"))
            b_parts.append(np.asfortranarray(b).ravel(order="F"))
            self.shapes.append((n, nr, xo))
            ao += n * n
            bo += n * nr
            xo += n * nr
        self.A = torch.from_numpy(np.concatenate(a_parts)).to(dev)
        self.B = torch.from_numpy(np.concatenate(b_parts)).to(dev)
        self.X = torch.zeros(xo, dtype=torch.float64, device=dev)
        raw = bytes(descs)
        self.desc = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
        self.res = torch.zeros(self.count * ctypes.sizeof(Result), dtype=torch.uint8, device=dev)
        ws = int(lib().ada_batched_workspace_size(self.count))
        self.work = torch.empty(ws, dtype=torch.uint8, device=dev)
        self.opts = make_opts(no_approx, rcond_threshold, LAYOUT_DENSE, 0, 0, force_general, want_berr, precision,
                              extensions)
        self.ctx = ctx or context(dev.index or 0)

    def run(self):
        import torch
        stream = torch.cuda.current_stream(self.A.device).cuda_stream
        rc = lib().ada_solve_batched(self.ctx.handle, self.count, self.desc.data_ptr(), self.A.data_ptr(),
                                     self.B.data_ptr(), self.X.data_ptr(), self.work.data_ptr(), self.work.numel(),
                                     ctypes.byref(self.opts), self.res.data_ptr(), ctypes.c_void_p(stream))
        if rc != OK:
            raise AdaError(rc, last_error())

    def tune(self):
        """ada_autotune_batched on this batch: the fastest launch shape is kept in the context for this
        precision (and X, results hold the solution). Returns (shape dict, ms per batch)."""
        import torch
        stream = torch.cuda.current_stream(self.A.device).cuda_stream
        out = BatchedShape()
        ms = ctypes.c_double()
        rc = lib().ada_autotune_batched(self.ctx.handle, self.count, self.desc.data_ptr(), self.A.data_ptr(),
                                        self.B.data_ptr(), self.X.data_ptr(), self.work.data_ptr(),
                                        self.work.numel(), ctypes.byref(self.opts), self.res.data_ptr(),
                                        ctypes.c_void_p(stream), ctypes.byref(out), ctypes.byref(ms))
        if rc != OK:
            raise AdaError(rc, last_error())
        return out.as_dict(), ms.value

    def set_shape(self, shape: "BatchedShape | None"):
        """ada_set_batched_shape for this batch's precision (None: the default shape)."""
        rc = lib().ada_set_batched_shape(self.ctx.handle, self.opts.precision,
                                         ctypes.byref(shape) if shape is not None else None)
        if rc != OK:
            raise AdaError(rc, last_error())

    def shape(self) -> dict:
        out = BatchedShape()
        rc = lib().ada_get_batched_shape(self.ctx.handle, self.opts.precision, ctypes.byref(out))
        if rc != OK:
            raise AdaError(rc, last_error())
        return out.as_dict()

    def results(self):
        raw = bytes(self.res.cpu().numpy().tobytes())
        arr = (Result * self.count).from_buffer_copy(raw)
        return [_result(r, r.status) for r in arr]

    def solutions(self):
        xs = self.X.cpu().numpy()
        return [xs[o:o + n * nr].reshape((n, nr), order="F") for (n, nr, o) in self.shapes]


def solve_batched(As, Bs, **kw):
    """Solve the systems A_k X_k = B_k (host arrays) with one batched launch; returns (Xs, results)."""
    import torch
    b = Batch(As, Bs, **kw)
    b.run()
    torch.cuda.synchronize()
    return b.solutions(), b.results()


class Server:
    """Continuous-batching solve server over a device arena (ada_server_*).

    submit() queues a request and returns its ticket at once; poll() waits for it.
    The tensors of a request are held until it has been polled to completion."""

    def __init__(self, arena_bytes: int, device="cuda:0", solve_workers: int = 3, ctx: Context | None = None):
        import torch
        dev = torch.device(device)
        self.device = dev
        self.ctx = ctx or context(dev.index or 0)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        rc = lib().ada_server_create(self.ctx.handle, self.arena.data_ptr(), self.arena.numel(), int(solve_workers),
                                     ctypes.byref(h))
        if rc != OK:
            raise AdaError(rc, last_error())
        self.handle = h
        self._held = {}

    def submit(self, A=None, B=None, X=None, *, keep=False, reuse=0, **opt_kw) -> int:
        """A: (n, n) float64 CUDA tensor (None with reuse), B: (n,) or (n, nrhs); X: output
        (allocated when None). Returns the ticket."""
        import torch
        Bc = _colmajor(B if B.dim() == 2 else B[:, None])
        n, nrhs = Bc.shape
        if X is None:
            X = torch.empty((nrhs, n), dtype=torch.float64, device=Bc.device).t()
        r = Request()
        r.n = 0 if reuse else n
        r.nrhs = nrhs
        r.ldb = Bc.stride(1) if nrhs > 1 else n
        r.ldx = X.stride(1) if nrhs > 1 else n
        r.keep_factor = int(keep)
        r.reuse = int(reuse)
        r.B = Bc.data_ptr()
        r.X = X.data_ptr()
        Ac = None
        if not reuse:
            Ac = _colmajor(A)
            r.A = Ac.data_ptr()
            r.lda = Ac.stride(1) if n > 1 else n
        r.opts = make_opts(**opt_kw) if opt_kw else Opts()
        t = ctypes.c_uint64()
        rc = lib().ada_submit(self.handle, ctypes.byref(r), ctypes.byref(t))
        if rc != OK:
            raise AdaError(rc, last_error())
        self._held[t.value] = (Ac, Bc, X)
        return t.value

    def poll(self, ticket: int, timeout_us: int = -1):
        """Returns None while pending, else (status, SolveResult, X, kept_factor, queue_us, total_us)."""
        res = Result()
        kept = ctypes.c_uint64()
        q = ctypes.c_double()
        tot = ctypes.c_double()
        rc = lib().ada_poll_timed(self.handle, ctypes.c_uint64(ticket), ctypes.byref(res), ctypes.byref(kept),
                                  int(timeout_us), ctypes.byref(q), ctypes.byref(tot))
        if rc == PENDING:
            return None
        if ticket not in self._held:
            raise AdaError(rc, last_error())
        _, _, X = self._held.pop(ticket)
        return rc, _result(res, rc), X, kept.value, q.value, tot.value

    def release(self, factor: int):
        rc = lib().ada_factor_release(self.handle, ctypes.c_uint64(factor))
        if rc != OK:
            raise AdaError(rc, last_error())

    def usage(self):
        used = ctypes.c_size_t()
        queued = ctypes.c_int()
        kept = ctypes.c_int()
        lib().ada_server_usage(self.handle, ctypes.byref(used), ctypes.byref(queued), ctypes.byref(kept))
        return used.value, queued.value, kept.value

    def close(self):
        if getattr(self, "handle", None):
            lib().ada_server_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
