"""Block orthonormalization of tall-skinny matrices on AMD MI355X (gfx950).

Python face of ``libborth.so`` (C ABI in ``include/borth.h``).  The method is
the two-phase orthogonalization of Sec. 4.2 of Alvermann et al. (arXiv
1806.01036): project X against a locked orthonormal basis Y, then
orthonormalize the result through its Gram matrix (CholQR / SVQB), iterated
(CholQR2); the first Gram matrix can be accumulated in double-double or as
split BF16 products on the matrix cores.

Tensors are torch CUDA (HIP) tensors, row-major with unit column stride; the
work is enqueued on torch's current stream.  Names mirror the C ABI.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _lib

__all__ = [
    "BorthError", "Breakdown", "Context", "Info", "default_context", "gram", "factor",
    "update", "orthonormalize", "orthonormalize_noalloc", "orthonormalize_dd", "stream_probe", "valu_probe",
    "orthonormalize_iter",
    "batch_orthonormalize", "GRAM", "FACT",
    "SCHED",
]

# "dd": DD Gram with the biased accumulation; "dd_dot2": DD Gram with Dot2
# (borth_gram's BORTH_GRAM_DD_DOT2, elsewhere BORTH_GRAM_DD + BORTH_FLAG_DD_DOT2)
GRAM = {"f64": 0, "dd": 1, "split": 2, "dd_dot2": 3}
FACT = {"chol": 0, "svqb": 1}
SCHED = {"auto": 0, "materialize": 1, "recompute": 2}
FLAG_SYNC, FLAG_PROJECT_ONCE, FLAG_GRAPH, FLAG_NO_FUSE, FLAG_RANK_REVEAL = 1, 2, 4, 8, 16
FLAG_DD_DOT2, FLAG_AUTO_ESCALATE, FLAG_BATCH_PERSISTENT = 32, 64, 128
OK, ERR_ARG, ERR_HIP, ERR_NOMEM, BREAKDOWN, NONFINITE, UNSUPPORTED = range(7)


class BorthError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"borth status {status}: {msg}")
        self.status = status


class Breakdown(BorthError):
    pass


class ArgumentError(BorthError, ValueError):
    """An argument the binding rejects before calling the library (the
    library's own checks report the same status, ERR_ARG)."""

    def __init__(self, msg):
        super().__init__(ERR_ARG, msg)


@dataclass
class Info:
    status: int
    failed_pass: int
    failed_pivot: int
    passes_run: int
    orth_est: float = 0.0   # ||R_p - I||_F of the last pass
    kappa_est: float = 0.0  # condition estimate from the first pass's factor
    escalation: int = 0     # escalate=True: 0 none, 1 DD Gram, 2 shifted DD
    svqb_lifted: int = 0    # SVQB: most eigenvalues one pass lifted to its floor


def _info(i):
    return Info(i.status, i.failed_pass, i.failed_pivot, i.passes_run, i.orth_est, i.kappa_est,
                i.escalation, i.svqb_lifted)


def _torch():
    import torch
    return torch


def _stream_handle():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A library context bound to one device (and torch's current stream)."""

    def __init__(self, device: int = 0):
        lib = _lib.load()
        h = ctypes.c_void_p()
        st = lib.borth_create(ctypes.byref(h), int(device), _stream_handle())
        if st != OK:
            raise BorthError(st, "borth_create failed")
        self.h = h
        self.device = device
        self.lib = lib

    def sync_stream(self):
        self.lib.borth_set_stream(self.h, _stream_handle())

    def check(self, st):
        if st == OK:
            return
        msg = self.lib.borth_last_error(self.h).decode()
        if st == BREAKDOWN:
            raise Breakdown(st, msg or "Cholesky breakdown")
        raise BorthError(st, msg or self.lib.borth_status_string(st).decode())

    def close(self):
        if self.h:
            self.lib.borth_destroy(self.h)
            self.h = None

    def set_profiling(self, on, kinds=(0, 1)):
        """Time the launches of ``kinds`` (0: first-pass Gram sweeps, 1:
        update sweeps) with HIP events; ``on=False`` stops."""
        mask = sum(1 << k for k in kinds) if on else 0
        self.check(self.lib.borth_set_profiling(self.h, mask))

    def kernel_time(self, kind: int):
        avg = ctypes.c_double()
        n = ctypes.c_int()
        self.check(self.lib.borth_kernel_time(self.h, kind, ctypes.byref(avg), ctypes.byref(n)))
        return avg.value, n.value

    def info(self) -> Info:
        inf = _lib.borth_info()
        self.check(self.lib.borth_get_info(self.h, ctypes.byref(inf)))
        return _info(inf)

    def autotune(self, cache_path=None, budget_ms=2000):
        p = None if cache_path is None else str(cache_path).encode()
        self.check(self.lib.borth_autotune(self.h, p, int(budget_ms)))

    def autotune_load(self, cache_path):
        self.check(self.lib.borth_autotune_load(self.h, str(cache_path).encode()))


_contexts = {}


def default_context(device=None) -> Context:
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _contexts:
        _contexts[dev] = Context(dev)
    ctx = _contexts[dev]
    ctx.sync_stream()
    return ctx


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _ld(t):
    if t is None:
        return 0
    if t.dim() != 2 or t.stride(1) != 1:
        raise ArgumentError("matrices must be 2-D and row-major (unit column stride; "
                            "use .contiguous())")
    return t.stride(0)


def _mat(t, name, ctx, rows=None, cols=None, f32=False, packed=False):
    """Check a matrix before its pointer goes to the library, which can
    check nothing about device memory: a 2-D tensor on the context's device,
    float64 (or float32 where ``f32``), unit column stride, leading dimension
    >= columns, the expected shape; ``packed``: a contiguous rows x cols
    array (R, C, Z and the Gram matrices have no leading dimension)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dim() != 2:
        raise ArgumentError(f"{name}: a 2-D tensor is required")
    if t.device.type != "cuda" or t.device.index != ctx.device:
        raise ArgumentError(f"{name}: must be on cuda:{ctx.device}, got {t.device}")
    if not (t.dtype == torch.float64 or (f32 and t.dtype == torch.float32)):
        raise ArgumentError(f"{name}: float64{' or float32' if f32 else ''} required, got {t.dtype}")
    if (rows is not None and t.shape[0] != rows) or (cols is not None and t.shape[1] != cols):
        raise ArgumentError(f"{name}: shape {tuple(t.shape)}, expected ({rows}, {cols})")
    if packed:
        if not t.is_contiguous():
            raise ArgumentError(f"{name}: must be contiguous")
    elif t.shape[1] > 1 and t.stride(1) != 1 or t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise ArgumentError(f"{name}: must be row-major (unit column stride, ld >= columns; "
                            "use .contiguous())")
    return t


def _outs(ctx, Q, R, C, m, k, ky):
    _mat(Q, "out", ctx, m, k)
    _mat(R, "R", ctx, k, k, packed=True)
    if ky:
        _mat(C, "C", ctx, ky, k, packed=True)


def _dt(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return 0
    if t.dtype == torch.float32:
        return 1
    raise ArgumentError("float64 or float32 tensors only")


def gram(B, A=None, prec="f64", ctx=None):
    """G = [A | B]^T [A | B] (hi, lo); lo is None unless prec is 'dd' or 'dd_dot2'."""
    torch = _torch()
    ctx = ctx or default_context(B.device.index)
    _mat(B, "B", ctx, f32=True)
    m, kb = B.shape
    if A is not None:
        _mat(A, "A", ctx, rows=m)
    ka = 0 if A is None else A.shape[1]
    W = ka + kb
    ghi = torch.empty((W, W), dtype=torch.float64, device=B.device)
    glo = (torch.empty((W, W), dtype=torch.float64, device=B.device)
           if prec in ("dd", "dd_dot2") else None)
    ctx.check(ctx.lib.borth_gram(ctx.h, m, ka, _ptr(A), _ld(A) if A is not None else ka, kb,
                                 _dt(B), _ptr(B), _ld(B), GRAM[prec], _ptr(ghi), _ptr(glo)))
    return ghi, glo


def factor(G_hi, G_lo=None, ky=0, fact="chol", shift=0.0, ctx=None, check=True):
    """Phase-II transform from the Gram matrix of [Y | X]: returns
    (Z, R, C, Info) with Z^T M Z = I."""
    torch = _torch()
    ctx = ctx or default_context(G_hi.device.index)
    W = G_hi.shape[0]
    _mat(G_hi, "G_hi", ctx, W, W, packed=True)
    if G_lo is not None:
        _mat(G_lo, "G_lo", ctx, W, W, packed=True)
    k = W - ky
    dev = G_hi.device
    Z = torch.zeros((k, k), dtype=torch.float64, device=dev)
    R = torch.zeros((k, k), dtype=torch.float64, device=dev)
    C = torch.zeros((max(ky, 1), k), dtype=torch.float64, device=dev)
    inf = _lib.borth_info()
    st = ctx.lib.borth_factor(ctx.h, ky, k, _ptr(G_hi), _ptr(G_lo), FACT[fact], float(shift),
                              _ptr(Z), _ptr(R), _ptr(C) if ky else ctypes.c_void_p(0),
                              ctypes.byref(inf))
    info = _info(inf)
    if check:
        ctx.check(st)
    return Z, R, C[:ky], info


def update(X, Z, Y=None, C=None, dense=False, out=None, ctx=None):
    """Q = (X - Y C) Z (binary64 result)."""
    torch = _torch()
    ctx = ctx or default_context(X.device.index)
    _mat(X, "X", ctx, f32=True)
    m, k = X.shape
    _mat(Z, "Z", ctx, k, k, packed=True)
    ky = 0 if Y is None else Y.shape[1]
    if ky:
        _mat(Y, "Y", ctx, rows=m)
        if C is None:
            raise ArgumentError("C is required with Y")
        _mat(C, "C", ctx, ky, k, packed=True)
    Q = out if out is not None else torch.empty((m, k), dtype=torch.float64, device=X.device)
    _mat(Q, "out", ctx, m, k)
    ctx.check(ctx.lib.borth_update(ctx.h, m, k, _dt(X), _ptr(X), _ld(X), _ptr(Y),
                                   _ld(Y) if ky else 0, ky, _ptr(C), _ptr(Z), int(bool(dense)),
                                   _ptr(Q), _ld(Q)))
    return Q


def _opts(gram, fact, passes, sched, shift, flags):
    o = _lib.borth_opts()
    o.gram = GRAM[gram]
    if gram == "dd_dot2":
        o.gram = GRAM["dd"]
        flags |= FLAG_DD_DOT2
    o.fact = FACT[fact]
    o.passes = int(passes)
    o.sched = SCHED[sched]
    o.shift = float(shift)
    o.flags = int(flags)
    return o


def orthonormalize(X, Y=None, *, gram="dd", fact="chol", passes=2, sched="auto", shift=-1.0,
                   project_once=False, graph=False, escalate=False, out=None, R=None, C=None,
                   sync=True, check=True, ctx=None):
    """X = Y C + Q R with Q^T Q = I and Y^T Q = 0.  Returns (Q, R, C, Info);
    Info is None when ``sync`` is False (the call is then fully asynchronous).
    ``escalate``: after a breakdown, repeat with the DD Gram, then with a
    shifted DD first pass and three passes (synchronizes)."""
    torch = _torch()
    ctx = ctx or default_context(X.device.index)
    _mat(X, "X", ctx, f32=True)
    m, k = X.shape
    ky = 0 if Y is None else Y.shape[1]
    if ky:
        _mat(Y, "Y", ctx, rows=m)
    dev = X.device
    Q = out if out is not None else torch.empty((m, k), dtype=torch.float64, device=dev)
    R = R if R is not None else torch.empty((k, k), dtype=torch.float64, device=dev)
    if ky and C is None:
        C = torch.empty((ky, k), dtype=torch.float64, device=dev)
    _outs(ctx, Q, R, C, m, k, ky)
    flags = ((FLAG_PROJECT_ONCE if project_once else 0) | (FLAG_GRAPH if graph else 0)
             | (FLAG_AUTO_ESCALATE if escalate else 0))
    o = _opts(gram, fact, passes, sched, shift, flags)
    inf = _lib.borth_info()
    st = ctx.lib.borth_orthonormalize(ctx.h, m, k, _dt(X), _ptr(X), _ld(X), _ptr(Y),
                                      _ld(Y) if ky else 0, ky, _ptr(Q), _ld(Q), _ptr(R),
                                      _ptr(C) if ky else ctypes.c_void_p(0), ctypes.byref(o),
                                      ctypes.byref(inf) if sync else None)
    info = _info(inf) if sync else None
    if check or st not in (BREAKDOWN, NONFINITE):
        ctx.check(st)
    return Q, R, (C if ky else None), info


def stream_probe(kind, src, dst, nbytes=None, reps=10, ctx=None):
    """HBM streaming probe (borth_stream_probe): kind "read", "copy" or
    "copy_nt" over ``nbytes`` (default: all of ``src``) of the device tensors
    ``src`` and ``dst``.  Returns (ms per launch, GB/s of the bytes moved,
    grid)."""
    ctx = ctx or default_context(src.device.index)
    k = {"read": 0, "copy": 1, "copy_nt": 2}[kind]
    n = int(nbytes if nbytes is not None else src.numel() * src.element_size())
    if not (src.is_cuda and dst.is_cuda) or n > src.numel() * src.element_size():
        raise ArgumentError("stream_probe: device tensors, nbytes within src")
    if k and n > dst.numel() * dst.element_size():
        raise ArgumentError("stream_probe: dst smaller than nbytes")
    if not k and dst.numel() * dst.element_size() < 65536:
        raise ArgumentError("stream_probe: a read needs 64 KiB of dst for its workgroup words")
    ms = ctypes.c_double()
    grid = ctypes.c_int()
    ctx.check(ctx.lib.borth_stream_probe(ctx.h, k, _ptr(src), _ptr(dst), n, int(reps),
                                         ctypes.byref(ms), ctypes.byref(grid)))
    moved = n * (1 if k == 0 else 2)
    return ms.value, moved / (ms.value * 1e-3) / 1e9, grid.value


def valu_probe(kind, sink, ctx=None):
    """FP64 vector-ALU probe (borth_valu_probe): kind "fma" (plain FMA
    chains) or "dd_step" (the DD Gram's fma, add, fma, add step) in registers,
    on the device tensor ``sink`` (at least 8 x 256 doubles per compute unit).
    Returns (FP64 lane operations per second, waves per SIMD of the fastest
    launch)."""
    ctx = ctx or default_context(sink.device.index)
    k = {"fma": 0, "dd_step": 1}[kind]
    if not sink.is_cuda:
        raise ArgumentError("valu_probe: sink must be a device tensor")
    rate = ctypes.c_double()
    waves = ctypes.c_int()
    ctx.check(ctx.lib.borth_valu_probe(ctx.h, k, _ptr(sink), sink.numel() * sink.element_size(),
                                       ctypes.byref(rate), ctypes.byref(waves)))
    return rate.value, waves.value


def orthonormalize_noalloc(X, Y=None, *, gram="dd", fact="chol", passes=2, sched="auto",
                           shift=-1.0, project_once=False, out=None, R=None, C=None, sync=True,
                           check=True, ctx=None):
    """borth_orthonormalize_noalloc: the same result as ``orthonormalize``
    with every workspace of the call in the library's per-device scratch
    array (the library allocates nothing in the call).  Calls that overlap
    on one GPU share that array and race.  Q, R and C must be given or are
    allocated here by torch, before the library is called."""
    torch = _torch()
    ctx = ctx or default_context(X.device.index)
    _mat(X, "X", ctx, f32=True)
    m, k = X.shape
    ky = 0 if Y is None else Y.shape[1]
    if ky:
        _mat(Y, "Y", ctx, rows=m)
    dev = X.device
    Q = out if out is not None else torch.empty((m, k), dtype=torch.float64, device=dev)
    R = R if R is not None else torch.empty((k, k), dtype=torch.float64, device=dev)
    if ky and C is None:
        C = torch.empty((ky, k), dtype=torch.float64, device=dev)
    _outs(ctx, Q, R, C, m, k, ky)
    o = _opts(gram, fact, passes, sched, shift, FLAG_PROJECT_ONCE if project_once else 0)
    inf = _lib.borth_info()
    st = ctx.lib.borth_orthonormalize_noalloc(
        ctx.h, m, k, _dt(X), _ptr(X), _ld(X), _ptr(Y), _ld(Y) if ky else 0, ky, _ptr(Q), _ld(Q),
        _ptr(R), _ptr(C) if ky else ctypes.c_void_p(0), ctypes.byref(o),
        ctypes.byref(inf) if sync else None)
    info = _info(inf) if sync else None
    if check or st not in (BREAKDOWN, NONFINITE):
        ctx.check(st)
    return Q, R, (C if ky else None), info


def orthonormalize_dd(X, Y=None, *, X_lo=None, fact="chol", dot2=False, out=None, out_lo=None,
                      R=None, C=None, check=True, ctx=None):
    """One DD pass (k <= 64) returning the result in double-double:
    (Q, Q_lo, R, C, Info) with Q + Q_lo the DD Q (borth_orthonormalize_dd).
    ``X_lo``: low words of a DD input X + X_lo (same shape and strides;
    k <= 32 and ky + k <= 64)."""
    torch = _torch()
    ctx = ctx or default_context(X.device.index)
    _mat(X, "X", ctx)
    m, k = X.shape
    ky = 0 if Y is None else Y.shape[1]
    if ky:
        _mat(Y, "Y", ctx, rows=m)
    dev = X.device
    Q = out if out is not None else torch.empty((m, k), dtype=torch.float64, device=dev)
    Ql = out_lo if out_lo is not None else torch.empty((m, k), dtype=torch.float64, device=dev)
    _mat(Ql, "out_lo", ctx, m, k)
    if X_lo is not None:
        _mat(X_lo, "X_lo", ctx, m, k)
    if _ld(Ql) != _ld(Q):
        raise ArgumentError("Q and Q_lo need the same leading dimension")
    if X_lo is not None and (X_lo.shape != X.shape or _ld(X_lo) != _ld(X)):
        raise ArgumentError("X_lo needs the shape and leading dimension of X")
    R = R if R is not None else torch.empty((k, k), dtype=torch.float64, device=dev)
    if ky and C is None:
        C = torch.empty((ky, k), dtype=torch.float64, device=dev)
    _outs(ctx, Q, R, C, m, k, ky)
    o = _opts("dd_dot2" if dot2 else "dd", fact, 1, "materialize", 0.0, 0)
    inf = _lib.borth_info()
    st = ctx.lib.borth_orthonormalize_dd(ctx.h, m, k, _ptr(X), _ptr(X_lo), _ld(X), _ptr(Y),
                                         _ld(Y) if ky else 0, ky, _ptr(Q), _ptr(Ql), _ld(Q),
                                         _ptr(R), _ptr(C) if ky else None, ctypes.byref(o),
                                         ctypes.byref(inf))
    if check or st not in (BREAKDOWN, NONFINITE):
        ctx.check(st)
    return Q, Ql, R, (C if ky else None), _info(inf)


@dataclass
class IterInfo:
    converged: bool
    passes_run: int
    c_norm: float
    r_dev: float
    rank: int = 0


def orthonormalize_iter(X, Y=None, *, gram="f64", fact="chol", eps=1e-10, max_iter=5, out=None,
                        R=None, C=None, fuse=True, B=None, rank_reveal=False, check=True,
                        ctx=None):
    """Iterated two-phase scheme: passes of projection against Y and
    orthonormalization until ||C_j||_F <= eps and ||R_j - I||_F <= eps (or
    max_iter passes).  ``fuse=False``: a full Gram sweep in every pass
    instead of Gram columns accumulated by the previous update.  ``B``: the
    diagonal of an SPD B (device vector of m weights) for the B-inner
    product.  ``rank_reveal`` (SVQB): drop the null directions of each pass
    (Q's first IterInfo.rank columns span the block, the rest are zero).
    Returns (Q, R, C, IterInfo, Info)."""
    torch = _torch()
    ctx = ctx or default_context(X.device.index)
    _mat(X, "X", ctx, f32=True)
    m, k = X.shape
    ky = 0 if Y is None else Y.shape[1]
    if ky:
        _mat(Y, "Y", ctx, rows=m)
    dev = X.device
    Q = out if out is not None else torch.empty((m, k), dtype=torch.float64, device=dev)
    R = R if R is not None else torch.empty((k, k), dtype=torch.float64, device=dev)
    if ky and C is None:
        C = torch.empty((ky, k), dtype=torch.float64, device=dev)
    _outs(ctx, Q, R, C, m, k, ky)
    o = _opts(gram, fact, 1, "materialize", 0.0,
              (0 if fuse else FLAG_NO_FUSE) | (FLAG_RANK_REVEAL if rank_reveal else 0))
    it = _lib.borth_iter_info()
    inf = _lib.borth_info()
    if B is None:
        st = ctx.lib.borth_orthonormalize_iter(
            ctx.h, m, k, _ptr(X), _ld(X), _ptr(Y), _ld(Y) if ky else 0, ky, _ptr(Q), _ld(Q),
            _ptr(R), _ptr(C) if ky else None, ctypes.byref(o), float(eps), int(max_iter),
            ctypes.byref(it), ctypes.byref(inf))
    else:
        if (B.dim() != 1 or B.shape[0] != m or B.dtype != torch.float64 or not B.is_contiguous()
                or B.device.type != "cuda" or B.device.index != ctx.device):
            raise ArgumentError(f"B must be a contiguous float64 vector of m weights on cuda:{ctx.device}")
        st = ctx.lib.borth_orthonormalize_iter_b(
            ctx.h, m, k, _ptr(X), _ld(X), _ptr(Y), _ld(Y) if ky else 0, ky, _ptr(B), _ptr(Q),
            _ld(Q), _ptr(R), _ptr(C) if ky else None, ctypes.byref(o), float(eps), int(max_iter),
            ctypes.byref(it), ctypes.byref(inf))
    if check or st not in (BREAKDOWN, NONFINITE):
        ctx.check(st)
    return (Q, R, (C if ky else None),
            IterInfo(bool(it.converged), it.passes_run, it.c_norm, it.r_dev, it.rank),
            _info(inf))


def batch_orthonormalize(blocks, *, gram="dd", fact="chol", passes=2, shift=-1.0,
                         project_once=False, graph=False, persistent=False, sync=True,
                         check=True, ctx=None):
    """Orthonormalize many independent blocks together (borth_batch_orthonormalize).

    blocks: list of dicts with X (m x k float64), optional Y (m x ky, ky <= 16)
    and optional preallocated Q (may be X itself: in place), R, C.  Each
    phase runs as one launch over all blocks, or with persistent=True (where
    every block fits it, see borth_batch_orthonormalize) the whole batch as
    one persistent launch; with graph=True the launch sequence is captured
    once and replayed.  Returns the list of (Q, R, C) and the list
    of Info (None entries when not synchronizing)."""
    torch = _torch()
    if not blocks:
        return [], []
    ctx = ctx or default_context(blocks[0]["X"].device.index)
    arr = (_lib.borth_block * len(blocks))()
    outs = []
    for i, b in enumerate(blocks):
        X = _mat(b["X"], f"blocks[{i}].X", ctx)
        Y = b.get("Y")
        m, k = X.shape
        ky = 0 if Y is None else Y.shape[1]
        if ky:
            _mat(Y, f"blocks[{i}].Y", ctx, rows=m)
        Q = b.get("Q")
        if Q is None:
            Q = torch.empty((m, k), dtype=torch.float64, device=X.device)
        Rt = b.get("R")
        if Rt is None:
            Rt = torch.empty((k, k), dtype=torch.float64, device=X.device)
        Ct = b.get("C")
        if ky and Ct is None:
            Ct = torch.empty((ky, k), dtype=torch.float64, device=X.device)
        _mat(Q, f"blocks[{i}].Q", ctx, m, k)
        _mat(Rt, f"blocks[{i}].R", ctx, k, k, packed=True)
        if ky:
            _mat(Ct, f"blocks[{i}].C", ctx, ky, k, packed=True)
        e = arr[i]
        e.m, e.k, e.X, e.ldx = m, k, X.data_ptr(), _ld(X)
        e.Y, e.ldy, e.ky = (Y.data_ptr() if ky else None), (_ld(Y) if ky else 0), ky
        e.Q, e.ldq, e.R = Q.data_ptr(), _ld(Q), Rt.data_ptr()
        e.C = Ct.data_ptr() if ky else None
        outs.append((Q, Rt, Ct if ky else None))
    flags = ((FLAG_PROJECT_ONCE if project_once else 0) | (FLAG_GRAPH if graph else 0)
             | (FLAG_BATCH_PERSISTENT if persistent else 0))
    o = _opts(gram, fact, passes, "materialize", shift, flags)
    infs = (_lib.borth_info * len(blocks))()
    st = ctx.lib.borth_batch_orthonormalize(ctx.h, len(blocks), arr, ctypes.byref(o),
                                            infs if sync else None)
    infos = [_info(i) for i in infs] \
        if sync else [None] * len(blocks)
    if check or st not in (BREAKDOWN, NONFINITE):
        ctx.check(st)
    return outs, infos
