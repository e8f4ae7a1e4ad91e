"""Python binding of libcur (maximal-volume CUR selection on MI355X).

Argument marshalling only: every step of the selection, assembly and residual
runs in the HIP library ``libcur.so`` built from ``csrc/``.  torch provides
device memory and the current HIP stream; no torch operator runs on the path.
Importing works without a GPU (the library loads, its symbols resolve);
calling a compute function without the built library or without a GPU raises.

Functions mirror the C ABI of ``include/cur.h``:
  select(A, r, ...)            -> dict(I, J, status, rank, nodes, phases, refreshes, swaps, logvol)
  assemble(A, I, J)            -> (C, U, R)
  residual(A, C, U, R, prec)   -> (cheb, fro_rel)
  select_batched(As, rs, ...)  -> list of (I, J, status)
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcur.so")

OK, WARN_NOCONV = 0, 1
ERR_ARG, ERR_RANK, ERR_NONFINITE, ERR_DEVICE, ERR_NOMEM, ERR_INTERNAL = -1, -2, -3, -4, -5, -6
METHOD_MAXVOL, METHOD_GREEDY = 0, 1
F64, F32 = 0, 1
PREC_NATIVE, PREC_BF16X3, PREC_FP8 = 0, 1, 2
TRACE_FIELDS = ("level", "index", "q", "short", "promoted", "nocap", "swaps", "phases",
                "refreshes", "vol_e")

EXPORTS = ("cur_opts_init", "cur_create", "cur_destroy", "cur_strerror", "cur_last_error",
           "cur_select", "cur_assemble", "cur_residual", "cur_select_batched",
           "cur_profile_enable", "cur_profile_read", "cur_tune_export", "cur_tune_import",
           "cur_residual_noalloc", "cur_mlp_features", "cur_mlp_forward", "cur_mlp_grad", "cur_mlp_adam")
NOALLOC_SCRATCH_BYTES = 16 << 20
MLP_FEATURES, MLP_HIDDEN, MLP_PARAMS, MLP_BLOB_BYTES = 4, 128, 17281, 35328


class CurError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class Trace(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int32), ("count", ctypes.c_int32),
                ("meta", ctypes.c_void_p), ("vol_mant", ctypes.c_void_p),
                ("I", ctypes.c_void_p), ("J", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("col_block", ctypes.c_int32),
                ("tau", ctypes.c_double), ("max_swaps", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("propose", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("mlp", ctypes.c_void_p), ("seed", ctypes.c_uint64),
                ("trace", ctypes.POINTER(Trace)), ("method", ctypes.c_int32), ("polish", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("nodes", ctypes.c_int32), ("phases", ctypes.c_int32),
                ("refreshes", ctypes.c_int32), ("swaps", ctypes.c_int64), ("logvol", ctypes.c_double)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("key", ctypes.c_int64 * 6), ("ms", ctypes.c_double * 3), ("tried", ctypes.c_int32),
                ("groups", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("busy", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("bytes", ctypes.c_double), ("fresh_launches", ctypes.c_int64), ("fresh_busy", ctypes.c_int64),
                ("fresh_seconds", ctypes.c_double), ("fresh_bytes", ctypes.c_double),
                ("bytes_inplace", ctypes.c_double), ("fresh_bytes_inplace", ctypes.c_double),
                ("busy_seconds", ctypes.c_double), ("fresh_busy_seconds", ctypes.c_double)]


class Item(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("r", ctypes.c_int32), ("A", ctypes.c_void_p),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("I", ctypes.c_void_p), ("J", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libcur.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2502_11017_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.cur_opts_init.argtypes = [ctypes.POINTER(Opts)]
        L.cur_opts_init.restype = None
        L.cur_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
        L.cur_create.restype = ctypes.c_int
        L.cur_destroy.argtypes = [P]
        L.cur_destroy.restype = ctypes.c_int
        L.cur_strerror.argtypes = [ctypes.c_int]
        L.cur_strerror.restype = ctypes.c_char_p
        L.cur_last_error.argtypes = []
        L.cur_last_error.restype = ctypes.c_char_p
        L.cur_select.argtypes = [P, ctypes.c_int, P, i64, i64, i64, i32, ctypes.POINTER(Opts), P, P,
                                 ctypes.POINTER(Info)]
        L.cur_select.restype = ctypes.c_int
        L.cur_assemble.argtypes = [P, ctypes.c_int, P, i64, i64, i64, i32, P, P, P, P, P]
        L.cur_assemble.restype = ctypes.c_int
        L.cur_residual.argtypes = [P, ctypes.c_int, P, i64, i64, i64, i32, P, P, P, i32,
                                   ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
        L.cur_residual.restype = ctypes.c_int
        L.cur_select_rect.argtypes = [P, ctypes.c_int, P, i64, i64, i64, i32, i32, ctypes.POINTER(Opts), P, P,
                                      ctypes.POINTER(Info)]
        L.cur_select_rect.restype = ctypes.c_int
        L.cur_assemble_rect.argtypes = [P, ctypes.c_int, P, i64, i64, i64, i32, i32, P, P, P, P, P]
        L.cur_assemble_rect.restype = ctypes.c_int
        L.cur_residual_rect.argtypes = [P, ctypes.c_int, P, i64, i64, i64, i32, i32, P, P, P,
                                        ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
        L.cur_residual_rect.restype = ctypes.c_int
        L.cur_residual_noalloc.argtypes = [P, ctypes.c_int, P, i64, i64, i64, i32, P, P, P, i32,
                                           ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
        L.cur_residual_noalloc.restype = ctypes.c_int
        L.cur_mlp_features.argtypes = [P, ctypes.c_int, P, i64, i64, i64, i32, i32, ctypes.c_uint64, P]
        L.cur_mlp_features.restype = ctypes.c_int
        L.cur_mlp_forward.argtypes = [P, P, P, i64, P]
        L.cur_mlp_forward.restype = ctypes.c_int
        L.cur_mlp_grad.argtypes = [P, P, P, P, i64, ctypes.c_float, P, ctypes.POINTER(dbl)]
        L.cur_mlp_grad.restype = ctypes.c_int
        L.cur_mlp_adam.argtypes = [P, P, P, P, P, P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float]
        L.cur_mlp_adam.restype = ctypes.c_int
        L.cur_select_batched.argtypes = [P, i32, ctypes.POINTER(Item), ctypes.POINTER(Opts),
                                         ctypes.POINTER(ctypes.c_int)]
        L.cur_select_batched.restype = ctypes.c_int
        L.cur_profile_enable.argtypes = [P, ctypes.c_int]
        L.cur_profile_enable.restype = ctypes.c_int
        L.cur_profile_read.argtypes = [P, ctypes.POINTER(Profile)]
        L.cur_profile_read.restype = ctypes.c_int
        L.cur_tune_export.argtypes = [P, ctypes.POINTER(TuneEntry), i32, ctypes.POINTER(i32)]
        L.cur_tune_export.restype = ctypes.c_int
        L.cur_tune_import.argtypes = [P, ctypes.POINTER(TuneEntry), i32]
        L.cur_tune_import.restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().cur_last_error().decode()


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        raise CurError(rc, f"{lib().cur_strerror(rc).decode()}: {last_error()}")
    return rc


_ctx = {}


def _torch():
    import torch

    return torch


def context(device=None):
    """Per-(device, stream) library context, created on first use."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("libcur needs a HIP GPU; none is visible")
    dev = torch.cuda.current_device() if device is None else int(device)
    stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, stream)
    if key not in _ctx:
        c = ctypes.c_void_p()
        _check(lib().cur_create(ctypes.byref(c), dev, ctypes.c_void_p(stream)))
        _ctx[key] = c
    return _ctx[key]


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("A must be float64 or float32")


def _matrix(A):
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor (unit column stride)")
    if not A.is_cuda:
        raise ValueError("A must live on the GPU")
    return A.shape[0], A.shape[1], A.stride(0)


def make_opts(col_block=0, tau=0.0, max_swaps=0, prec=PREC_NATIVE, trace=None, groups=0, method=0,
              mlp=None, seed=0, polish=False) -> Opts:
    o = Opts()
    lib().cur_opts_init(ctypes.byref(o))
    o.groups = int(groups)
    o.method = int(method)
    o.polish = 1 if polish else 0
    if mlp is not None:  # a device tensor holding the weight blob: the learned proposal
        o.propose = 1
        o.mlp = ctypes.c_void_p(mlp.data_ptr())
        o.seed = int(seed)
    o.col_block = int(col_block)
    o.tau = float(tau)
    o.max_swaps = int(max_swaps)
    o.prec = int(prec)
    if trace is not None:
        o.trace = ctypes.pointer(trace)
    return o


def tree_size(n: int, w: int) -> int:
    c = max(1, n // w)
    tot = 0
    while True:
        tot += c
        if c <= 1:
            return tot
        c = (c + 1) // 2


def select(A, r: int, col_block: int = 0, tau: float = 0.0, max_swaps: int = 0, trace: bool = False,
           allow=(OK, WARN_NOCONV, ERR_RANK), groups: int = 0, method: int = METHOD_MAXVOL, mlp=None, seed: int = 0,
           polish: bool = False):
    """Select r rows I and r columns J of the device matrix A (cur_select);
    polish: then the swap loop once more over all columns (cur_opts.polish)."""
    torch = _torch()
    m, n, lda = _matrix(A)
    ctx = context(A.device.index)
    I = torch.empty(r, dtype=torch.int64, device=A.device)
    J = torch.empty(r, dtype=torch.int64, device=A.device)
    info = Info()
    tr = None
    host = None
    if trace:
        import numpy as np

        w = col_block if col_block else max(64, r)
        N = 1 if method == METHOD_GREEDY else tree_size(n, max(w, 1)) + (1 if polish else 0)
        host = {"meta": np.zeros((N, 10), dtype=np.int64), "vol_m": np.zeros(N),
                "I": np.zeros((N, r), dtype=np.int64), "J": np.zeros((N, r), dtype=np.int64)}
        tr = Trace(N, 0, host["meta"].ctypes.data, host["vol_m"].ctypes.data,
                   host["I"].ctypes.data, host["J"].ctypes.data)
    o = make_opts(col_block, tau, max_swaps, trace=tr, groups=groups, method=method, mlp=mlp, seed=seed,
                  polish=polish)
    rc = lib().cur_select(ctx, _dtype_code(A), ctypes.c_void_p(A.data_ptr()), m, n, lda, r,
                          ctypes.byref(o), ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(J.data_ptr()),
                          ctypes.byref(info))
    _check(rc, allow)
    out = {"I": I, "J": J, "status": rc, "rank": info.rank, "nodes": info.nodes,
           "phases": info.phases, "refreshes": info.refreshes, "swaps": info.swaps,
           "logvol": info.logvol}
    if trace:  # the records the library wrote (a polish over a rank-short root writes none)
        out["trace"] = {k: v[:tr.count] for k, v in host.items()}
    return out


def assemble(A, I, J):
    """C = A(:,J), U = A(I,J)^+ (FP64), R = A(I,:) (cur_assemble)."""
    torch = _torch()
    m, n, lda = _matrix(A)
    r = int(I.numel())
    ctx = context(A.device.index)
    C = torch.empty((m, r), dtype=A.dtype, device=A.device)
    U = torch.empty((r, r), dtype=torch.float64, device=A.device)
    R = torch.empty((r, n), dtype=A.dtype, device=A.device)
    I = I.to(torch.int64).contiguous()
    J = J.to(torch.int64).contiguous()
    rc = lib().cur_assemble(ctx, _dtype_code(A), ctypes.c_void_p(A.data_ptr()), m, n, lda, r,
                            ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(J.data_ptr()),
                            ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                            ctypes.c_void_p(R.data_ptr()))
    _check(rc)
    return C, U, R


def residual(A, C, U, R, prec: int = PREC_NATIVE):
    """(max|A - CUR|, ||A - CUR||_F / ||A||_F) (cur_residual)."""
    m, n, lda = _matrix(A)
    r = int(U.shape[0])
    ctx = context(A.device.index)
    C = C.contiguous()
    U = U.contiguous()
    R = R.contiguous()
    cheb = ctypes.c_double()
    fro = ctypes.c_double()
    rc = lib().cur_residual(ctx, _dtype_code(A), ctypes.c_void_p(A.data_ptr()), m, n, lda, r,
                            ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                            ctypes.c_void_p(R.data_ptr()), int(prec), ctypes.byref(cheb), ctypes.byref(fro))
    _check(rc)
    return cheb.value, fro.value


def select_rect(A, r: int, c: int, method: int = METHOD_MAXVOL, col_block: int = 0, tau: float = 0.0,
                max_swaps: int = 0, groups: int = 0, allow=(OK, WARN_NOCONV, ERR_RANK), polish: bool = False):
    """r rows I and c columns J chosen independently (Alg. 2), cur_select_rect;
    polish (r == c): then the swap loop on the cross over all columns."""
    torch = _torch()
    m, n, lda = _matrix(A)
    ctx = context(A.device.index)
    I = torch.empty(r, dtype=torch.int64, device=A.device)
    J = torch.empty(c, dtype=torch.int64, device=A.device)
    info = Info()
    o = make_opts(col_block, tau, max_swaps, groups=groups, method=method, polish=polish)
    rc = lib().cur_select_rect(ctx, _dtype_code(A), ctypes.c_void_p(A.data_ptr()), m, n, lda, r, c,
                               ctypes.byref(o), ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(J.data_ptr()),
                               ctypes.byref(info))
    _check(rc, allow)
    return {"I": I, "J": J, "status": rc, "rank": info.rank, "nodes": info.nodes, "phases": info.phases,
            "refreshes": info.refreshes, "swaps": info.swaps, "logvol": info.logvol}


def assemble_rect(A, I, J):
    """C = A(:,J) (m x c), U = A(I,J)^+ (c x r, FP64), R = A(I,:) (r x n), cur_assemble_rect."""
    torch = _torch()
    m, n, lda = _matrix(A)
    r, c = int(I.numel()), int(J.numel())
    ctx = context(A.device.index)
    C = torch.empty((m, c), dtype=A.dtype, device=A.device)
    U = torch.empty((c, r), dtype=torch.float64, device=A.device)
    R = torch.empty((r, n), dtype=A.dtype, device=A.device)
    I = I.to(torch.int64).contiguous()
    J = J.to(torch.int64).contiguous()
    rc = lib().cur_assemble_rect(ctx, _dtype_code(A), ctypes.c_void_p(A.data_ptr()), m, n, lda, r, c,
                                 ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(J.data_ptr()),
                                 ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                                 ctypes.c_void_p(R.data_ptr()))
    _check(rc)
    return C, U, R


def residual_rect(A, C, U, R):
    """(max|A - CUR|, ||A - CUR||_F / ||A||_F) of a rectangular cross, cur_residual_rect."""
    m, n, lda = _matrix(A)
    c, r = int(U.shape[0]), int(U.shape[1])
    ctx = context(A.device.index)
    C, U, R = C.contiguous(), U.contiguous(), R.contiguous()
    cheb, fro = ctypes.c_double(), ctypes.c_double()
    rc = lib().cur_residual_rect(ctx, _dtype_code(A), ctypes.c_void_p(A.data_ptr()), m, n, lda, r, c,
                                 ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                                 ctypes.c_void_p(R.data_ptr()), ctypes.byref(cheb), ctypes.byref(fro))
    _check(rc)
    return cheb.value, fro.value


def residual_noalloc(A, C, U, R, prec: int = PREC_NATIVE):
    """cur_residual_noalloc: the residual with every temporary in the library's
    fixed per-GPU scratch array (no device allocation; calls on one GPU must
    not overlap)."""
    m, n, lda = _matrix(A)
    r = int(U.shape[0])
    ctx = context(A.device.index)
    C = C.contiguous()
    U = U.contiguous()
    R = R.contiguous()
    cheb = ctypes.c_double()
    fro = ctypes.c_double()
    rc = lib().cur_residual_noalloc(ctx, _dtype_code(A), ctypes.c_void_p(A.data_ptr()), m, n, lda, r,
                                    ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                                    ctypes.c_void_p(R.data_ptr()), int(prec), ctypes.byref(cheb), ctypes.byref(fro))
    _check(rc)
    return cheb.value, fro.value


def mlp_features(A, r: int, col_block: int = 0, seed: int = 0):
    """Proposal features of every (leaf, row): float32 (b m, 4) on A's device."""
    torch = _torch()
    m, n, lda = _matrix(A)
    w = col_block if col_block else max(64, r)
    b = max(1, n // w)
    F = torch.empty((b * m, MLP_FEATURES), dtype=torch.float32, device=A.device)
    _check(lib().cur_mlp_features(context(A.device.index), _dtype_code(A), ctypes.c_void_p(A.data_ptr()), m, n, lda,
                                  int(r), int(col_block), int(seed), ctypes.c_void_p(F.data_ptr())))
    return F


def mlp_forward(blob, F):
    """Scores of the feature rows F (float32 (count, 4)) under the weight blob."""
    torch = _torch()
    F = F.contiguous()
    out = torch.empty(F.shape[0], dtype=torch.float32, device=F.device)
    _check(lib().cur_mlp_forward(context(F.device.index), ctypes.c_void_p(blob.data_ptr()),
                                 ctypes.c_void_p(F.data_ptr()), int(F.shape[0]), ctypes.c_void_p(out.data_ptr())))
    return out


def mlp_grad(blob, F, y, pos_weight: float = 1.0):
    """(gradient float32[MLP_PARAMS], mean loss) of the weighted logistic loss."""
    torch = _torch()
    F = F.contiguous()
    y = y.to(torch.float32).contiguous()
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=F.device)
    loss = ctypes.c_double()
    _check(lib().cur_mlp_grad(context(F.device.index), ctypes.c_void_p(blob.data_ptr()), ctypes.c_void_p(F.data_ptr()),
                              ctypes.c_void_p(y.data_ptr()), int(F.shape[0]), float(pos_weight),
                              ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss)))
    return g, loss.value


def mlp_adam(blob, params, m1, m2, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on params (float32[MLP_PARAMS], in place) that also writes the blob."""
    _check(lib().cur_mlp_adam(context(params.device.index), ctypes.c_void_p(blob.data_ptr()),
                              ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(m1.data_ptr()),
                              ctypes.c_void_p(m2.data_ptr()), ctypes.c_void_p(grad.data_ptr()), int(step), float(lr),
                              float(beta1), float(beta2), float(eps)))


def mlp_pack(params):
    """A weight blob (uint8 device tensor) holding the FP32 parameter vector params."""
    torch = _torch()
    blob = torch.zeros(MLP_BLOB_BYTES, dtype=torch.uint8, device=params.device)
    z = torch.zeros_like(params)
    p = params.clone()
    mlp_adam(blob, p, z.clone(), z.clone(), z, 1, 0.0)
    return blob


def profile_enable(enable=True, device=None):
    """Set the row-kernel timing / algorithmic-byte counters (cleared): False
    or 0 off, True or 1 the streaming pass kernel, 2 also the fresh kernel."""
    _check(lib().cur_profile_enable(context(device), int(enable)))


def profile_read(device=None) -> dict:
    p = Profile()
    _check(lib().cur_profile_read(context(device), ctypes.byref(p)))
    return {"launches": p.launches, "busy": p.busy, "seconds": p.seconds, "bytes": p.bytes,
            "bytes_inplace": p.bytes_inplace,
            "fresh_launches": p.fresh_launches, "fresh_busy": p.fresh_busy,
            "fresh_seconds": p.fresh_seconds, "fresh_bytes": p.fresh_bytes,
            "fresh_bytes_inplace": p.fresh_bytes_inplace,
            "busy_seconds": p.busy_seconds, "fresh_busy_seconds": p.fresh_busy_seconds}


def tune_export(device=None) -> list:
    """The context's launch-shape autotuner cache as a list of dicts."""
    ctx = context(device)
    n = ctypes.c_int32(0)
    _check(lib().cur_tune_export(ctx, None, 0, ctypes.byref(n)))
    buf = (TuneEntry * max(n.value, 1))()
    _check(lib().cur_tune_export(ctx, buf, n.value, ctypes.byref(n)))
    return [{"key": list(e.key), "ms": list(e.ms), "tried": e.tried, "groups": e.groups}
            for e in buf[:n.value]]


def tune_import(entries, device=None):
    """Replace the context's autotuner cache (entries as from tune_export)."""
    buf = (TuneEntry * max(len(entries), 1))()
    for k, e in enumerate(entries):
        buf[k] = TuneEntry((ctypes.c_int64 * 6)(*e["key"]), (ctypes.c_double * 3)(*e["ms"]),
                           int(e["tried"]), int(e["groups"]))
    _check(lib().cur_tune_import(context(device), buf, len(entries)))


def select_batched(As, rs, col_block: int = 0, tau: float = 0.0, max_swaps: int = 0, groups: int = 0,
                   polish: bool = False):
    """Independent selections of several device matrices (cur_select_batched);
    polish: each tree's root polished over all its matrix's columns."""
    torch = _torch()
    cnt = len(As)
    items = (Item * max(cnt, 1))()
    outs = []
    for k, (A, r) in enumerate(zip(As, rs)):
        m, n, lda = _matrix(A)
        I = torch.empty(r, dtype=torch.int64, device=A.device)
        J = torch.empty(r, dtype=torch.int64, device=A.device)
        items[k] = Item(_dtype_code(A), int(r), A.data_ptr(), m, n, lda, I.data_ptr(), J.data_ptr())
        outs.append((I, J))
    per = (ctypes.c_int * max(cnt, 1))()
    o = make_opts(col_block, tau, max_swaps, groups=groups, polish=polish)
    ctx = context(As[0].device.index if cnt else None)
    rc = lib().cur_select_batched(ctx, cnt, items, ctypes.byref(o), per)
    _check(rc, (OK, WARN_NOCONV, ERR_RANK))
    return [(I, J, per[k]) for k, (I, J) in enumerate(outs)], rc
