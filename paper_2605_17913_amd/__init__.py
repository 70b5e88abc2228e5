"""Batched single-precision differentiable interior-point QP solver for
MI355X (gfx950).

Thin ctypes binding over ``libqpx.so`` (C-ABI in ``include/qpx.h``).  Every
step of the solver runs in the library's HIP kernels; PyTorch only provides
device memory and the current stream.  There is no CPU fallback: if the
library is missing or the tensors are not on a GPU, the calls raise.

    minimize 1/2 x'Qx + q'x  s.t.  A x = b,  G x <= h        (batched)

Main entry points
    solve(Q, q, A, b, G, h, ...)           -> dict(x, y, z, s, status, iters, res)
    backward(Q, q, A, b, G, h, sol, gx)    -> dict of gradients (relax + IFT)
    QPFunction / qp_layer                  torch.autograd wrapper
    Server                                 continuous-batching request loop
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# QPX_LIB selects another build of the same library (e.g. a profiling build)
LIB_PATH = os.environ.get("QPX_LIB") or os.path.join(_HERE, "libqpx.so")

QPX_OK, QPX_PENDING = 0, 1
CONVERGED, MAX_ITER, NONFINITE, FACTOR_FAIL = 0, 1, 2, 3
STAGES = ["none", "scaling", "predictor", "centering", "corrector", "linesearch", "relax", "backward"]
FORMS = {"bounded": 0, "standard": 1, "condensed": 2}
# H-block assembly arithmetic (qp_opts.assembly)
ASSEMBLY = {"auto": 0, "fp32": 1, "bf16x3": 2, "mfma_fp32": 3}
# residual precision (qp_opts.fp64_residual)
RESIDUAL = {"auto": 0, "fp64": 1, "fp32": 2}

_c_int32, _c_float, _vp = ctypes.c_int32, ctypes.c_float, ctypes.c_void_p


class _Batch(ctypes.Structure):
    _fields_ = [("B", _c_int32), ("n", _c_int32), ("m", _c_int32), ("p", _c_int32),
                ("Q", _vp), ("q", _vp), ("A", _vp), ("b", _vp), ("G", _vp), ("h", _vp)]


class _Opts(ctypes.Structure):
    _fields_ = [("form", _c_int32), ("max_iter", _c_int32), ("tol", _c_float),
                ("sigma", _c_float), ("pc", _c_int32), ("kappa_relax", _c_float),
                ("relax_max_iter", _c_int32), ("relax_tol", _c_float), ("kmax", _c_int32),
                ("delta_reg", _c_float), ("refine_steps", _c_int32), ("block", _c_int32),
                ("assembly", _c_int32), ("backoff", _c_float), ("fp64_residual", _c_int32)]


class _Out(ctypes.Structure):
    _fields_ = [("x", _vp), ("y", _vp), ("z", _vp), ("s", _vp), ("status", _vp),
                ("iters", _vp), ("res", _vp), ("work", _vp)]


class _Grads(ctypes.Structure):
    _fields_ = [("dQ", _vp), ("dq", _vp), ("dA", _vp), ("db", _vp), ("dG", _vp), ("dh", _vp)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("max_slots", _c_int32), ("iters_per_step", _c_int32), ("n_max", _c_int32),
                ("arena_bytes", ctypes.c_size_t)]


class _Timing(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("status", _c_int32), ("iters", _c_int32)]


class _Plan(ctypes.Structure):
    _fields_ = [("threads", _c_int32), ("kb", _c_int32), ("factor_in_lds", _c_int32),
                ("assembly", _c_int32), ("lds_bytes", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t)]


EXPORTS = ["qp_default_opts", "qp_create", "qp_destroy", "qp_solve", "qp_solve_noalloc",
           "qp_backward",
           "qp_status_string", "qp_result_string", "qp_plan_query", "qp_server_create", "qp_serve_submit", "qp_serve_poll",
           "qp_serve_stats", "qp_server_destroy"]

_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """Load libqpx.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2605_17913_amd.build` (no CPU fallback)")
            L = ctypes.CDLL(LIB_PATH)
            L.qp_default_opts.argtypes = [ctypes.POINTER(_Opts)]
            L.qp_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
            L.qp_destroy.argtypes = [_vp]
            L.qp_solve.argtypes = [_vp, ctypes.POINTER(_Batch), ctypes.POINTER(_Opts),
                                   ctypes.POINTER(_Out), _vp]
            L.qp_solve_noalloc.argtypes = [_vp, ctypes.POINTER(_Batch), ctypes.POINTER(_Opts),
                                           ctypes.POINTER(_Out), _vp]
            L.qp_backward.argtypes = [_vp, ctypes.POINTER(_Batch), ctypes.POINTER(_Opts),
                                      ctypes.POINTER(_Out), _vp, _vp, _vp,
                                      ctypes.POINTER(_Grads), ctypes.POINTER(_Out), _vp]
            L.qp_status_string.restype = ctypes.c_char_p
            L.qp_result_string.argtypes = [_c_int32]
            L.qp_result_string.restype = ctypes.c_char_p
            L.qp_plan_query.argtypes = [_c_int32, _c_int32, _c_int32, ctypes.POINTER(_Opts),
                                        ctypes.POINTER(_Plan)]
            L.qp_server_create.argtypes = [_vp, ctypes.POINTER(_ServerOpts), ctypes.POINTER(_Opts),
                                           ctypes.POINTER(_vp)]
            L.qp_serve_submit.argtypes = [_vp, _c_int32, _c_int32, _c_int32, _vp, _vp, _vp, _vp,
                                          _vp, _vp, ctypes.POINTER(ctypes.c_uint64)]
            L.qp_serve_poll.argtypes = [_vp, ctypes.c_uint64, _vp, _vp, _vp, _vp,
                                        ctypes.POINTER(_Timing)]
            L.qp_serve_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_c_int32)]
            L.qp_server_destroy.argtypes = [_vp]
            _lib = L
    return _lib


class QPError(RuntimeError):
    pass


def plan(n: int, m: int, p: int, **kw) -> dict:
    """Launch plan for one problem size (host only): threads per QP, border
    cap, whether the factor fits LDS, assembly arithmetic, LDS bytes and
    global workspace bytes per QP."""
    o = make_opts(**kw)
    pl = _Plan()
    _check(lib().qp_plan_query(n, m, p, ctypes.byref(o), ctypes.byref(pl)), "qp_plan_query")
    inv = {v: k for k, v in ASSEMBLY.items()}
    return {"threads": pl.threads, "kb": pl.kb, "factor_in_lds": bool(pl.factor_in_lds),
            "assembly": inv[pl.assembly], "lds_bytes": pl.lds_bytes,
            "workspace_bytes": pl.workspace_bytes}


def _check(rc: int, what: str):
    if rc != QPX_OK:
        msg = lib().qp_status_string(rc).decode()
        raise QPError(f"{what} failed: {msg} ({rc})")


_ctx = {}


def _context(device: int):
    if device not in _ctx:
        h = _vp()
        _check(lib().qp_create(ctypes.byref(h), device), "qp_create")
        _ctx[device] = h
    return _ctx[device]


def default_opts() -> _Opts:
    o = _Opts()
    lib().qp_default_opts(ctypes.byref(o))
    return o


def make_opts(form="bounded", tol=None, max_iter=None, sigma=None, pc=None, kappa_relax=None,
              relax_max_iter=None, relax_tol=None, kmax=None, delta_reg=None, refine_steps=None,
              block=None, assembly=None, backoff=None, residual=None) -> _Opts:
    """qp_opts with the library defaults, overridden by the given values.
    assembly: "auto" | "fp32" | "bf16x3" | "mfma_fp32"; residual (the
    fp64_residual field): "auto" | "fp64" | "fp32"."""
    o = default_opts()
    o.form = FORMS[form] if isinstance(form, str) else int(form)
    if assembly is not None:
        o.assembly = ASSEMBLY[assembly] if isinstance(assembly, str) else int(assembly)
    if residual is not None:
        o.fp64_residual = RESIDUAL[residual] if isinstance(residual, str) else int(residual)
    for k, v in dict(tol=tol, max_iter=max_iter, sigma=sigma, kappa_relax=kappa_relax,
                     relax_max_iter=relax_max_iter, relax_tol=relax_tol, kmax=kmax,
                     delta_reg=delta_reg, refine_steps=refine_steps, block=block,
                     backoff=backoff).items():
        if v is not None:
            setattr(o, k, v)
    if pc is not None:
        o.pc = int(bool(pc))
    return o


def _ptr(t):
    return None if t is None or t.numel() == 0 else ctypes.c_void_p(t.data_ptr())


def _prep(t, shape, device, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise QPError(f"{name} must be a GPU tensor (no CPU path)")
    if t.device.index != device:
        raise QPError(f"{name} is on another device")
    t = t.to(torch.float32).contiguous()
    if tuple(t.shape) != tuple(shape):
        raise QPError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _batch(Q, q, A, b, G, h):
    if Q.dim() != 3:
        raise QPError("Q must be [B, n, n]")
    B, n = Q.shape[0], Q.shape[1]
    dev = Q.device.index if Q.device.type == "cuda" else -1
    if dev < 0:
        raise QPError("tensors must be on the GPU (no CPU path)")
    p = 0 if A is None else A.shape[1]
    m = 0 if G is None else G.shape[1]
    Q = _prep(Q, (B, n, n), dev, "Q")
    q = _prep(q, (B, n), dev, "q")
    A = _prep(A, (B, p, n), dev, "A") if p else None
    b = _prep(b, (B, p), dev, "b") if p else None
    G = _prep(G, (B, m, n), dev, "G") if m else None
    h = _prep(h, (B, m), dev, "h") if m else None
    st = _Batch(B, n, m, p, _ptr(Q), _ptr(q), _ptr(A), _ptr(b), _ptr(G), _ptr(h))
    return st, (Q, q, A, b, G, h), (B, n, m, p, dev)


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def solve(Q, q, A, b, G, h, *, opts: _Opts | None = None, work: bool = False, **kw):
    """Solve a batch of QPs on the GPU (Algorithm 1, or the standard IPM
    with form="standard").  Returns a dict of tensors x, y, z, s, status,
    iters, res (and work = algorithmic flops per QP if requested)."""
    st, keep, (B, n, m, p, dev) = _batch(Q, q, A, b, G, h)
    o = opts if opts is not None else make_opts(**kw)
    f32 = dict(dtype=torch.float32, device=Q.device)
    out = dict(x=torch.empty(B, n, **f32), y=torch.empty(B, p, **f32),
               z=torch.empty(B, m, **f32), s=torch.empty(B, m, **f32),
               status=torch.empty(B, dtype=torch.int32, device=Q.device),
               iters=torch.empty(B, dtype=torch.int32, device=Q.device),
               res=torch.empty(B, **f32))
    if work:
        out["work"] = torch.empty(B, dtype=torch.float64, device=Q.device)
    so = _Out(_ptr(out["x"]), _ptr(out["y"]), _ptr(out["z"]), _ptr(out["s"]),
              _ptr(out["status"]), _ptr(out["iters"]), _ptr(out["res"]),
              _ptr(out.get("work")))
    _check(lib().qp_solve(_context(dev), ctypes.byref(st), ctypes.byref(o), ctypes.byref(so),
                          _stream(dev)), "qp_solve")
    return out


def solve_noalloc(Q, q, A, b, G, h, out, *, opts: _Opts | None = None, **kw):
    """qp_solve_noalloc: solve into the caller's preallocated output tensors
    `out` (dict with x [B,n], y [B,p], z [B,m], s [B,m], status int32 [B] and
    optionally iters int32 [B], res float32 [B]); the call allocates no
    device memory (factors that do not fit LDS use the library's fixed
    per-device workspace of NOALLOC_SCRATCH_BYTES).  Raises QPError if the
    batch needs more workspace than that."""
    st, keep, (B, n, m, p, dev) = _batch(Q, q, A, b, G, h)
    o = opts if opts is not None else make_opts(**kw)
    so = _Out(_ptr(out["x"]), _ptr(out.get("y")), _ptr(out.get("z")), _ptr(out.get("s")),
              _ptr(out["status"]), _ptr(out.get("iters")), _ptr(out.get("res")), None)
    _check(lib().qp_solve_noalloc(_context(dev), ctypes.byref(st), ctypes.byref(o),
                                  ctypes.byref(so), _stream(dev)), "qp_solve_noalloc")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def backward(Q, q, A, b, G, h, sol, dl_dx, dl_dy=None, dl_dz=None, *, opts: _Opts | None = None,
             relaxed: bool = False, work: bool = False, **kw):
    """Relax the solution to kappa_relax (Algorithm 2), factor there and
    return the parameter gradients of Algorithm 3 (dQ, dq, dA, db, dG, dh)."""
    st, keep, (B, n, m, p, dev) = _batch(Q, q, A, b, G, h)
    o = opts if opts is not None else make_opts(**kw)
    gx = _prep(dl_dx, (B, n), dev, "dl_dx")
    gy = _prep(dl_dy, (B, p), dev, "dl_dy") if (dl_dy is not None and p) else None
    gz = _prep(dl_dz, (B, m), dev, "dl_dz") if (dl_dz is not None and m) else None
    xs = _prep(sol["x"], (B, n), dev, "x")
    ys = _prep(sol["y"], (B, p), dev, "y") if p else None
    zs = _prep(sol["z"], (B, m), dev, "z") if m else None
    ss = _prep(sol["s"], (B, m), dev, "s") if m else None
    f32 = dict(dtype=torch.float32, device=Q.device)
    g = dict(Q=torch.empty(B, n, n, **f32), q=torch.empty(B, n, **f32),
             A=torch.empty(B, p, n, **f32), b=torch.empty(B, p, **f32),
             G=torch.empty(B, m, n, **f32), h=torch.empty(B, m, **f32))
    sg = _Grads(_ptr(g["Q"]), _ptr(g["q"]), _ptr(g["A"]), _ptr(g["b"]), _ptr(g["G"]), _ptr(g["h"]))
    so = _Out(_ptr(xs), _ptr(ys), _ptr(zs), _ptr(ss), None, None, None, None)
    rel = None
    ro = None
    if relaxed or work:
        rel = dict(x=torch.empty(B, n, **f32), y=torch.empty(B, p, **f32),
                   z=torch.empty(B, m, **f32), s=torch.empty(B, m, **f32),
                   status=torch.empty(B, dtype=torch.int32, device=Q.device),
                   iters=torch.empty(B, dtype=torch.int32, device=Q.device),
                   res=torch.empty(B, **f32),
                   work=torch.empty(B, dtype=torch.float64, device=Q.device))
        ro = _Out(_ptr(rel["x"]), _ptr(rel["y"]), _ptr(rel["z"]), _ptr(rel["s"]),
                  _ptr(rel["status"]), _ptr(rel["iters"]), _ptr(rel["res"]), _ptr(rel["work"]))
    _check(lib().qp_backward(_context(dev), ctypes.byref(st), ctypes.byref(o), ctypes.byref(so),
                             _ptr(gx), _ptr(gy), _ptr(gz), ctypes.byref(sg),
                             ctypes.byref(ro) if ro is not None else None, _stream(dev)),
           "qp_backward")
    if rel is not None:
        g["relaxed"] = rel
    return g


class QPFunction(torch.autograd.Function):
    """x* = argmin QP(Q, q, A, b, G, h) as a differentiable function of the
    problem data (paper sections 2.3 and 5): the forward pass is Algorithm 1,
    the backward pass relaxes to kappa_relax (Algorithm 2) and applies the
    implicit-function-theorem product of Algorithm 3, all in the library's
    kernels.  A, b (p = 0) and G, h (m = 0) may be None.  Returns (x, status);
    status (int32 [B], not differentiable) is the per-QP status word of the
    solve.  With check=True a QP that did not converge in the solve, or
    whose relaxation did not converge in the backward pass, raises QPError.
    `options` is a dict of make_opts keyword arguments."""

    @staticmethod
    def forward(ctx, Q, q, A, b, G, h, options, check):
        options = dict(options or {})
        sol = solve(Q, q, A, b, G, h, **options)
        status = sol["status"]
        if check:
            bad = torch.nonzero((status & 0xFF) != 0).flatten()
            if bad.numel():
                raise QPError(f"{bad.numel()} QP(s) did not converge in the solve, first "
                              f"{bad[0].item()}: {result_string(int(status[bad[0]].item()))}")
        ctx.options = options
        ctx.check = check
        ctx.has_A, ctx.has_G = A is not None, G is not None
        ctx.dtypes = [None if t is None else t.dtype for t in (Q, q, A, b, G, h)]
        ctx.save_for_backward(Q, q, A, b, G, h, sol["x"], sol["y"], sol["z"], sol["s"])
        ctx.mark_non_differentiable(status)
        return sol["x"], status

    @staticmethod
    def backward(ctx, gx, _gstatus):
        Q, q, A, b, G, h, x, y, z, s = ctx.saved_tensors
        need = ctx.needs_input_grad[:6]
        if not any(need):
            return (None,) * 8
        g = backward(Q, q, A, b, G, h, dict(x=x, y=y, z=z, s=s),
                     gx.to(torch.float32).contiguous(), relaxed=ctx.check, **ctx.options)
        if ctx.check:
            rst = g["relaxed"]["status"]
            bad = torch.nonzero((rst & 0xFF) != 0).flatten()
            if bad.numel():
                raise QPError(f"{bad.numel()} QP(s) did not converge in the relaxation, first "
                              f"{bad[0].item()}: {result_string(int(rst[bad[0]].item()))}")
        out = []
        for k, key in enumerate(("Q", "q", "A", "b", "G", "h")):
            present = ctx.dtypes[k] is not None
            out.append(g[key].to(ctx.dtypes[k]) if (present and need[k]) else None)
        return (*out, None, None)


def qp_layer(Q, q, A=None, b=None, G=None, h=None, *, return_status=False, check=True,
             **options):
    """Differentiable batched QP layer: x*(Q, q, A, b, G, h) (see QPFunction).
    return_status=True also returns the per-QP status words."""
    x, status = QPFunction.apply(Q, q, A, b, G, h, options, check)
    return (x, status) if return_status else x


def result_string(status: int) -> str:
    """Human-readable description of a per-QP status word."""
    return lib().qp_result_string(int(status)).decode()


class Server:
    """Continuous-batching request loop (C-ABI qp_server_*).  Requests are
    single QPs given as host float32 arrays; results come back as numpy
    arrays with host monotonic timestamps."""

    def __init__(self, device: int = 0, max_slots: int = 256, iters_per_step: int = 4,
                 n_max: int = 256, arena_bytes: int = 0, **solver_opts):
        import numpy as np  # noqa: F401
        self._np = np
        so = make_opts(**solver_opts)
        o = _ServerOpts(max_slots, iters_per_step, n_max, arena_bytes)
        h = _vp()
        _check(lib().qp_server_create(_context(device), ctypes.byref(o), ctypes.byref(so),
                                      ctypes.byref(h)), "qp_server_create")
        self._h = h
        self._sizes = {}

    def submit(self, Q, q, A, b, G, h) -> int:
        np = self._np
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
        Q, q, A, b, G, h = (f(a) for a in (Q, q, A, b, G, h))
        n = Q.shape[0]
        p = 0 if A is None else A.shape[0]
        m = 0 if G is None else G.shape[0]
        ptr = lambda a: None if a is None or a.size == 0 else a.ctypes.data_as(_vp)
        t = ctypes.c_uint64()
        _check(lib().qp_serve_submit(self._h, n, m, p, ptr(Q), ptr(q), ptr(A), ptr(b), ptr(G),
                                     ptr(h), ctypes.byref(t)), "qp_serve_submit")
        self._sizes[t.value] = (n, m, p)
        return t.value

    def poll(self, ticket: int):
        np = self._np
        n, m, p = self._sizes[ticket]
        x, y = np.empty(n, np.float32), np.empty(p, np.float32)
        z, s = np.empty(m, np.float32), np.empty(m, np.float32)
        tm = _Timing()
        ptr = lambda a: None if a.size == 0 else a.ctypes.data_as(_vp)
        rc = lib().qp_serve_poll(self._h, ticket, ptr(x), ptr(y), ptr(z), ptr(s), ctypes.byref(tm))
        if rc == QPX_PENDING:
            return None
        _check(rc, "qp_serve_poll")
        del self._sizes[ticket]
        return dict(x=x, y=y, z=z, s=s, status=tm.status, iters=tm.iters,
                    t_submit=tm.t_submit, t_admit=tm.t_admit, t_done=tm.t_done)

    def wait(self, ticket: int, timeout: float = 60.0, sleep: float = 2e-4):
        import time
        t0 = time.monotonic()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() - t0 > timeout:
                raise QPError(f"request {ticket} not done after {timeout} s")
            time.sleep(sleep)

    def stats(self):
        a, c, pk = ctypes.c_uint64(), ctypes.c_uint64(), _c_int32()
        _check(lib().qp_serve_stats(self._h, ctypes.byref(a), ctypes.byref(c), ctypes.byref(pk)),
               "qp_serve_stats")
        return dict(admitted=a.value, completed=c.value, peak_resident=pk.value)

    def close(self):
        if self._h is not None:
            lib().qp_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
