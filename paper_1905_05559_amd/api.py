"""Python binding of the C ABI (include/hess.h) over torch device tensors.

Only argument marshalling happens here: every step of the computation runs in
the HIP kernels of libhess.so.  torch provides device memory and the stream.
The function names follow the C entry points.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import torch

from . import _lib as L


class HessError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (L.STATUS_NAMES.get(status, str(status)), msg))
        self.status = status
        self.name = L.STATUS_NAMES.get(status, str(status))


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.float64:
        return 0
    if t == torch.float32:
        return 1
    raise TypeError("only float32 / float64 arrays are accepted, got %s" % t)


class Context:
    """A library context bound to one device and one stream, plus a grow-only workspace."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.lib = L.load()
        self.device = int(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = self.lib.hess_create(C.byref(h), self.device, C.c_void_p(self.stream.cuda_stream))
        if st != L.HESS_OK:
            raise HessError(st, "hess_create failed")
        self.h = h
        self._ws: Optional[torch.Tensor] = None

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8,
                                   device="cuda:%d" % self.device)
        return self._ws

    def release_workspace(self):
        self._ws = None

    def set_option(self, name: str, value: int):
        self._check(self.lib.hess_set_option(self.h, L.OPT[name], int(value)))

    def mfma_stream_rate(self, kind: str, iters: int = 20000) -> float:
        """Sustained TFLOP/s of one MFMA instruction in a register-only stream (hess_diag.h).
        kind: "f32_16x16x4", "bf16_16x16x32", "bf16_32x32x16" or "f64_16x16x4"."""
        k = {"f32_16x16x4": 0, "bf16_16x16x32": 1, "bf16_32x32x16": 2, "f64_16x16x4": 3}[kind]
        sink = torch.empty(1, dtype=torch.float32, device="cuda:%d" % self.device)
        out = C.c_double()
        self._check(self.lib.hess_mfma_stream_rate(self.h, k, int(iters), C.c_void_p(sink.data_ptr()), C.byref(out)))
        return out.value

    def autotune_report(self) -> str:
        """The autotuning decisions of this context (see hess_autotune_report)."""
        need = C.c_size_t()
        self._check(self.lib.hess_autotune_report(self.h, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        self._check(self.lib.hess_autotune_report(self.h, buf, need.value, None))
        return buf.value.decode()

    def profile(self) -> dict:
        """Per-kernel-class aggregates {name: {launches, ms, flops, bytes}} since the last reset."""
        buf = (L.HessProfEntry * 64)()
        n = self.lib.hess_profile_read(self.h, buf, 64)
        return {buf[i].name.decode(): {"launches": buf[i].launches, "ms": buf[i].ms, "flops": buf[i].flops,
                                       "bytes": buf[i].bytes} for i in range(min(n, 64))}

    def profile_reset(self):
        self._check(self.lib.hess_profile_reset(self.h))

    def last_error(self) -> str:
        return self.lib.hess_last_error(self.h).decode()

    def _check(self, st: int):
        if st != L.HESS_OK:
            raise HessError(st, self.last_error())

    def close(self):
        if self.h:
            self.lib.hess_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_DEFAULT = {}


def default_context(device: int = 0) -> Context:
    if device not in _DEFAULT:
        _DEFAULT[device] = Context(device)
    return _DEFAULT[device]


class MLP:
    """Weights W^(l-1) (T_l x T_{l-1}) and biases b^(l) as device tensors (Sec. 2)."""

    def __init__(self, T: Sequence[int], acts: Sequence[str], W: List[torch.Tensor], b: List[torch.Tensor]):
        self.T = [int(t) for t in T]
        self.acts = list(acts)
        self.W = [w.contiguous() for w in W]
        self.b = [v.contiguous() for v in b]
        assert len(self.acts) == len(self.T) - 2
        assert len(self.W) == len(self.T) - 1 and len(self.b) == len(self.T) - 1
        self.dtype = self.W[0].dtype
        for k in range(len(self.T) - 1):
            assert tuple(self.W[k].shape) == (self.T[k + 1], self.T[k])
            assert tuple(self.b[k].shape) == (self.T[k + 1],)
            assert self.W[k].dtype == self.dtype and self.b[k].dtype == self.dtype

    @property
    def P(self) -> int:
        return sum(self.T[k + 1] * self.T[k] + self.T[k + 1] for k in range(len(self.T) - 1))

    @classmethod
    def from_workload(cls, w, device="cuda:0", dtype: Optional[torch.dtype] = None):
        cv = lambda a: torch.from_numpy(a).to(device=device, dtype=dtype) if dtype else torch.from_numpy(a).to(device)
        return cls(w.T, w.acts, [cv(x) for x in w.W], [cv(x) for x in w.b])

    def struct(self):
        n = len(self.T)
        T = (C.c_int64 * n)(*self.T)
        act = (C.c_int32 * max(1, n - 2))(*[L.ACT[a] for a in self.acts])
        Wp = (C.c_void_p * (n - 1))(*[w.data_ptr() for w in self.W])
        bp = (C.c_void_p * (n - 1))(*[v.data_ptr() for v in self.b])
        s = L.HessMlp(n, T, act, _dtype_code(self.dtype), Wp, bp)
        s._keep = (T, act, Wp, bp)
        return s


def _data(X: torch.Tensor, Y: torch.Tensor) -> L.HessData:
    X = X.contiguous()
    Y = Y.contiguous()
    assert X.dtype == Y.dtype and X.shape[0] == Y.shape[0]
    d = L.HessData(int(X.shape[0]), _dtype_code(X.dtype), X.data_ptr(), Y.data_ptr())
    d._keep = (X, Y)
    return d


def _out_dtype(prec: str) -> torch.dtype:
    return torch.float64 if prec == "f64" else torch.float32


def workspace_size(op: str, model: MLP, X=None, Y=None, prec: str = "f32", arg: int = 0, opts=None,
                   ctx: Optional[Context] = None) -> int:
    ctx = ctx or default_context()
    m = model.struct() if model is not None else None
    d = _data(X, Y) if X is not None else None
    nb = C.c_size_t()
    ctx._check(ctx.lib.hess_workspace_size(ctx.h, L.OP[op], C.byref(m) if m else None,
                                           C.byref(d) if d else None, L.PREC[prec], int(arg),
                                           C.byref(opts) if opts is not None else None, C.byref(nb)))
    return nb.value


def hess_opg(model: MLP, X: torch.Tensor, Y: torch.Tensor, prec: str = "f32",
             out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """OPG = J^T J / N (P x P), see hess_opg in include/hess.h."""
    ctx = ctx or default_context()
    P = model.P
    if out is None:
        out = torch.empty((P, P), dtype=_out_dtype(prec), device=X.device)
    m, d = model.struct(), _data(X, Y)
    nb = workspace_size("opg", model, X, Y, prec, ctx=ctx)
    ws = ctx.workspace(nb)
    ctx._check(ctx.lib.hess_opg(ctx.h, C.byref(m), C.byref(d), L.PREC[prec], out.data_ptr(),
                                ws.data_ptr(), ws.numel()))
    return out


def hess_exact(model: MLP, X: torch.Tensor, Y: torch.Tensor, prec: str = "f32",
               out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Exact Hessian H (P x P), see hess_exact in include/hess.h."""
    ctx = ctx or default_context()
    P = model.P
    if out is None:
        out = torch.empty((P, P), dtype=_out_dtype(prec), device=X.device)
    m, d = model.struct(), _data(X, Y)
    nb = workspace_size("exact", model, X, Y, prec, ctx=ctx)
    ws = ctx.workspace(nb)
    ctx._check(ctx.lib.hess_exact(ctx.h, C.byref(m), C.byref(d), L.PREC[prec], out.data_ptr(),
                                  ws.data_ptr(), ws.numel()))
    return out


def hess_hvp(model: MLP, X: torch.Tensor, Y: torch.Tensor, V: torch.Tensor, prec: str = "f32",
             out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """H V for the rows of V (B x P), see hess_hvp in include/hess.h."""
    ctx = ctx or default_context()
    V = V.contiguous()
    B = int(V.shape[0])
    if out is None:
        out = torch.empty_like(V)
    m, d = model.struct(), _data(X, Y)
    nb = workspace_size("hvp", model, X, Y, prec, arg=B, ctx=ctx)
    ws = ctx.workspace(nb)
    ctx._check(ctx.lib.hess_hvp(ctx.h, C.byref(m), C.byref(d), L.PREC[prec], B, V.data_ptr(),
                                out.data_ptr(), ws.data_ptr(), ws.numel()))
    return out


CURV_MODES = {"low_quad": 0, "full_quad": 1, "low_apply": 2, "full_apply": 3, "full_inverse": 4}


def curvature(mode: str, lam: torch.Tensor, Q: torch.Tensor, X: torch.Tensor, lam_tilde: Optional[float] = None,
              out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Low/full-rank curvature operator queries from K eigenpairs (hess_curvature in include/hess.h).
    lam (K,), Q (K x P), X (nx x P), all FP64 on the device; lam_tilde defaults to lam[-1]."""
    ctx = ctx or default_context()
    K, P = int(Q.shape[0]), int(Q.shape[1])
    X = X.contiguous()
    nx = int(X.shape[0])
    lt = float(lam[-1].item()) if lam_tilde is None else float(lam_tilde)
    m = CURV_MODES[mode]
    if out is None:
        shape = (nx,) if m in (0, 1) else (nx, P)
        out = torch.empty(shape, dtype=torch.float64, device=X.device)
    kk = C.c_int64(K)
    nb = C.c_size_t()
    ctx._check(ctx.lib.hess_workspace_size(ctx.h, L.OP["curvature"], None, None, L.PREC["f64"], nx, C.byref(kk),
                                           C.byref(nb)))
    ws = ctx.workspace(nb.value)
    ctx._check(ctx.lib.hess_curvature(ctx.h, m, K, P, lam.data_ptr(), Q.contiguous().data_ptr(), lt, nx,
                                      X.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel()))
    return out


def curvature_noalloc(mode: str, lam: torch.Tensor, Q: torch.Tensor, X: torch.Tensor,
                      lam_tilde: Optional[float] = None, out: Optional[torch.Tensor] = None,
                      ctx: Optional[Context] = None) -> torch.Tensor:
    """As curvature(), through hess_curvature_noalloc: no workspace argument, the library's
    own device scratch (include/hess.h).  `out` should be passed by callers that must not
    allocate; lam, Q and X must already be contiguous FP64 device tensors."""
    ctx = ctx or default_context()
    K, P = int(Q.shape[0]), int(Q.shape[1])
    nx = int(X.shape[0])
    if not (lam.is_contiguous() and Q.is_contiguous() and X.is_contiguous()):
        raise ValueError("curvature_noalloc takes contiguous lam, Q and X")
    lt = float(lam[-1].item()) if lam_tilde is None else float(lam_tilde)
    m = CURV_MODES[mode]
    if out is None:
        shape = (nx,) if m in (0, 1) else (nx, P)
        out = torch.empty(shape, dtype=torch.float64, device=X.device)
    ctx._check(ctx.lib.hess_curvature_noalloc(ctx.h, m, K, P, lam.data_ptr(), Q.data_ptr(), lt, nx,
                                              X.data_ptr(), out.data_ptr()))
    return out


def syev(A: torch.Tensor, ctx: Optional[Context] = None):
    """Eigen-decomposition of a symmetric FP64 device matrix (n <= 512; rows may be
    strided): returns (w descending (n,), U (n x n), row j = eigenvector j), see
    hess_syev in include/hess.h."""
    ctx = ctx or default_context()
    if A.dtype != torch.float64 or A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
        raise ValueError("syev takes a square FP64 matrix with unit column stride")
    n = int(A.shape[0])
    w = torch.empty(n, dtype=torch.float64, device=A.device)
    U = torch.empty((n, n), dtype=torch.float64, device=A.device)
    nb = C.c_size_t()
    ctx._check(ctx.lib.hess_workspace_size(ctx.h, L.OP["syev"], None, None, L.PREC["f64"], n, None, C.byref(nb)))
    ws = ctx.workspace(nb.value)
    ctx._check(ctx.lib.hess_syev(ctx.h, n, A.data_ptr(), int(A.stride(0)), w.data_ptr(), U.data_ptr(),
                                 ws.data_ptr(), ws.numel()))
    return w, U


class HvpOperator:
    """Prepared HVP operator of (model, X, Y): the per-example passes run once, then
    apply(V) forms H V for blocks of up to max_B directions (hess_hvp_prepare /
    hess_hvp_apply in include/hess.h).  Holds its own workspace until close()."""

    def __init__(self, model: MLP, X: torch.Tensor, Y: torch.Tensor, prec: str = "f32", max_B: int = 512,
                 ctx: Optional[Context] = None):
        self.ctx = ctx or default_context()
        self.prec, self.max_B, self.P = prec, int(max_B), model.P
        nb = workspace_size("hvp", model, X, Y, prec, arg=self.max_B, ctx=self.ctx)
        self.ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=X.device)
        m, d = model.struct(), _data(X, Y)
        h = C.c_void_p()
        self.ctx._check(self.ctx.lib.hess_hvp_prepare(self.ctx.h, C.byref(m), C.byref(d), L.PREC[prec], self.max_B,
                                                      self.ws.data_ptr(), self.ws.numel(), C.byref(h)))
        self.h = h

    def apply(self, V: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        V = V.contiguous()
        if out is None:
            out = torch.empty_like(V)
        self.ctx._check(self.ctx.lib.hess_hvp_apply(self.ctx.h, self.h, int(V.shape[0]), V.data_ptr(),
                                                    out.data_ptr()))
        return out

    def close(self):
        if self.h:
            self.ctx.lib.hess_hvp_release(self.h)
            self.h = None
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hess_exact_cols(model: MLP, X: torch.Tensor, Y: torch.Tensor, col0: int, ncols: int, prec: str = "f32",
                    out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Columns col0 .. col0+ncols-1 of H (P x ncols), see hess_exact_cols in include/hess.h."""
    ctx = ctx or default_context()
    if out is None:
        out = torch.empty((model.P, ncols), dtype=torch.float64 if prec == "f64" else torch.float32,
                          device=X.device)
    m, d = model.struct(), _data(X, Y)
    nb = workspace_size("exact_cols", model, X, Y, prec, arg=ncols, ctx=ctx)
    ws = ctx.workspace(nb)
    ctx._check(ctx.lib.hess_exact_cols(ctx.h, C.byref(m), C.byref(d), L.PREC[prec], int(col0), int(ncols),
                                       out.data_ptr(), ws.data_ptr(), ws.numel()))
    return out


def eig_opts(which: str = "H", source: str = "matrix_free", M: Optional[torch.Tensor] = None,
             prec: str = "f32", oversample: int = 10, max_iter: int = 200, tol: float = 1e-5,
             seed: int = 0, method: str = "subspace", block: int = 0) -> L.HessEigOpts:
    """Options of hess_topk_eig; method "subspace" (filtered subspace iteration) or
    "lanczos" (thick-restart block Lanczos with blocks of `block` vectors, 0 = 32)."""
    o = L.HessEigOpts()
    o.which = 0 if which == "H" else 1
    o.source = 0 if source == "matrix_free" else 1
    o.M = M.data_ptr() if M is not None else None
    o.M_dtype = _dtype_code(M.dtype) if M is not None else 0
    o.prec = L.PREC[prec]
    o.P = int(M.shape[0]) if M is not None else 0
    o.oversample = int(oversample)
    o.max_iter = int(max_iter)
    o.tol = float(tol)
    o.seed = int(seed)
    o.method = {"subspace": 0, "lanczos": 1}[method]
    o.block = int(block)
    o._keep = M
    return o


def hess_topk_eig(model: Optional[MLP], X: Optional[torch.Tensor], Y: Optional[torch.Tensor], K: int,
                  opts: L.HessEigOpts, ctx: Optional[Context] = None, device: str = "cuda:0",
                  raise_on_noconv: bool = True):
    """K algebraically largest eigenpairs: returns (lambda (K,), Q (K x P), info dict, status name)."""
    ctx = ctx or default_context()
    P = model.P if model is not None else int(opts.P)
    lam = torch.empty(K, dtype=torch.float64, device=device)
    Q = torch.empty((K, P), dtype=torch.float64, device=device)
    m = model.struct() if model is not None else None
    d = _data(X, Y) if X is not None else None
    nb = C.c_size_t()
    ctx._check(ctx.lib.hess_workspace_size(ctx.h, L.OP["topk"], C.byref(m) if m else None,
                                           C.byref(d) if d else None, opts.prec, int(K), C.byref(opts),
                                           C.byref(nb)))
    ws = ctx.workspace(nb.value)
    info = L.HessEigInfo()
    st = ctx.lib.hess_topk_eig(ctx.h, C.byref(m) if m else None, C.byref(d) if d else None, int(K),
                               C.byref(opts), lam.data_ptr(), Q.data_ptr(), C.byref(info), ws.data_ptr(),
                               ws.numel())
    if st != L.HESS_OK and not (st == 8 and not raise_on_noconv):
        raise HessError(st, ctx.last_error())
    inf = {"iters": info.iters, "applies": info.applies, "max_rel_residual": info.max_rel_residual,
           "shift_used": info.shift_used}
    return lam, Q, inf, L.STATUS_NAMES[st]


def hess_predvar(model: MLP, lam: torch.Tensor, Q: torch.Tensor, delta: float, Xq: torch.Tensor,
                 cls: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Damped curvature query s_q for the rows of Xq, see hess_predvar in include/hess.h."""
    ctx = ctx or default_context()
    Xq = Xq.contiguous()
    nq = int(Xq.shape[0])
    K = int(lam.shape[0])
    s = torch.empty(nq, dtype=torch.float64, device=Xq.device)
    m = model.struct()
    nb = C.c_size_t()
    ctx._check(ctx.lib.hess_workspace_size(ctx.h, L.OP["predvar"], C.byref(m), None, 0, nq, None,
                                           C.byref(nb)))
    ws = ctx.workspace(nb.value)
    ctx._check(ctx.lib.hess_predvar(ctx.h, C.byref(m), K, lam.data_ptr(), Q.data_ptr(), float(delta), nq,
                                    Xq.data_ptr(), cls.data_ptr() if cls is not None else None,
                                    s.data_ptr(), ws.data_ptr(), ws.numel()))
    return s


def batched_workspace_size(models: List[MLP], Xs: List[torch.Tensor], Ys: List[torch.Tensor],
                           ctx: Optional[Context] = None, prec: str = "f32") -> int:
    """Workspace bytes hess_batched needs for these networks (hess_workspace_size, op batched)."""
    ctx = ctx or default_context()
    M = len(models)
    ms = (L.HessMlp * M)()
    ds = (L.HessData * M)()
    keep = []
    for i, (m, X, Y) in enumerate(zip(models, Xs, Ys)):
        s = m.struct()
        d = _data(X, Y)
        keep.append((s, d))
        ms[i] = s
        ds[i] = d
    nb = C.c_size_t()
    ctx._check(ctx.lib.hess_workspace_size(ctx.h, L.OP["batched"], ms, ds, L.PREC[prec], M, None, C.byref(nb)))
    return nb.value


def hess_batched(models: List[MLP], Xs: List[torch.Tensor], Ys: List[torch.Tensor], with_H: bool = True,
                 with_G: bool = True, outs_H=None, outs_G=None, ctx: Optional[Context] = None, prec: str = "f32"):
    """Exact H and/or OPG (FP32; prec "f32" or "f32_split") of several networks in one call,
    see hess_batched in include/hess.h.

    Returns (list of H or None, list of G or None)."""
    ctx = ctx or default_context()
    M = len(models)
    ms = (L.HessMlp * M)()
    ds = (L.HessData * M)()
    keep = []
    for i, (m, X, Y) in enumerate(zip(models, Xs, Ys)):
        s = m.struct()
        d = _data(X, Y)
        keep.append((s, d))
        ms[i] = s
        ds[i] = d
    Hs = outs_H if outs_H is not None else ([torch.empty((m.P, m.P), dtype=torch.float32, device=Xs[0].device)
                                               for m in models] if with_H else None)
    Gs = outs_G if outs_G is not None else ([torch.empty((m.P, m.P), dtype=torch.float32, device=Xs[0].device)
                                               for m in models] if with_G else None)
    hp = (C.c_void_p * M)(*[h.data_ptr() for h in Hs]) if Hs is not None else None
    gp = (C.c_void_p * M)(*[g.data_ptr() for g in Gs]) if Gs is not None else None
    nb = C.c_size_t()
    ctx._check(ctx.lib.hess_workspace_size(ctx.h, L.OP["batched"], ms, ds, L.PREC[prec], M, None, C.byref(nb)))
    ws = ctx.workspace(nb.value)
    ctx._check(ctx.lib.hess_batched(ctx.h, M, ms, ds, L.PREC[prec], hp, gp, ws.data_ptr(), ws.numel()))
    return Hs, Gs


class Server:
    """Continuous-batching server of curvature requests (hess_server_* in include/hess.h).

    pool_bytes of device memory (a torch buffer owned by this object) back every
    request's workspace; n_slots worker slots run requests concurrently on their own
    streams; coalesce merges queued damped queries against the same target."""

    REQ = {"full": 0, "topk": 1, "predvar": 2, "curvature": 3}

    def __init__(self, pool_bytes: int, n_slots: int = 4, coalesce: bool = True, device: int = 0):
        self.lib = L.load()
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda:%d" % device)
        h = C.c_void_p()
        st = self.lib.hess_server_create(C.byref(h), device, int(n_slots), C.c_void_p(self.pool.data_ptr()),
                                         self.pool.numel(), 1 if coalesce else 0)
        if st != L.HESS_OK:
            raise HessError(st, "hess_server_create failed")
        self.h = h
        self._keep = {}

    def submit(self, kind: str, model: MLP, X=None, Y=None, H=None, G=None, K=0, lam=None, Q=None, tol=1e-5,
               seed=0, delta=0.0, Xq=None, cls=None, s=None, curv_mode=None, lam_tilde=0.0,
               fault_launch: int = 0) -> int:
        """Queue one request.  kind "curvature": lam, Q (K pairs), Xq = nq x P FP64 vectors,
        s = outputs (nq for the quadratic forms, nq x P for the products), curv_mode one of
        CURV_MODES, lam_tilde the full-rank level.  fault_launch > 0 (test hook) makes the
        request's n-th kernel launch report HESS_E_DEVICE without launching it."""
        r = L.HessRequest()
        r.kind = self.REQ[kind]
        m = model.struct()
        r.model = m
        keep = [m, model]
        if X is not None:
            d = _data(X, Y)
            r.data = d
            keep.append(d)
        r.H = H.data_ptr() if H is not None else None
        r.G = G.data_ptr() if G is not None else None
        r.K = int(K)
        r.lam = lam.data_ptr() if lam is not None else None
        r.Q = Q.data_ptr() if Q is not None else None
        r.tol = float(tol)
        r.seed = int(seed)
        r.delta = float(delta)
        if Xq is not None:
            r.nq = int(Xq.shape[0])
            r.Xq = Xq.data_ptr()
        r.cls = cls.data_ptr() if cls is not None else None
        r.s = s.data_ptr() if s is not None else None
        if kind == "curvature":
            if Xq is None or Xq.dtype != torch.float64 or not Xq.is_contiguous():
                raise ValueError("curvature requests take contiguous FP64 vectors Xq (nq x P)")
            r.curv_mode = CURV_MODES[curv_mode] if isinstance(curv_mode, str) else int(curv_mode)
            r.lam_tilde = float(lam_tilde)
        r.fault_launch = int(fault_launch)
        keep += [H, G, lam, Q, Xq, cls, s, X, Y]
        rid = C.c_uint64()
        st = self.lib.hess_server_submit(self.h, C.byref(r), C.byref(rid))
        if st != L.HESS_OK:
            raise HessError(st, "submit failed")
        self._keep[rid.value] = keep
        return rid.value

    def wait(self, rid: int):
        """Returns (status name, latency in ms)."""
        lat = C.c_double()
        st = self.lib.hess_server_wait(self.h, C.c_uint64(rid), C.byref(lat))
        self._keep.pop(rid, None)
        return L.STATUS_NAMES.get(st, str(st)), lat.value

    def stats(self) -> dict:
        a = (C.c_int64 * 4)()
        self.lib.hess_server_stats(self.h, a)
        return {"submitted": a[0], "completed": a[1], "failed": a[2], "coalesced_batches": a[3]}

    def close(self):
        if self.h:
            self.lib.hess_server_destroy(self.h)
            self.h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
