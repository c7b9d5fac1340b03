"""MOR-based adaptive parareal (arXiv 2601.10981) on MI355X.

Python binding of libpr.so (include/pr.h): the same entry points, taking
torch tensors for device memory and torch's current HIP stream. Every step of
the method runs in the library's HIP kernels; this module only marshals
arguments. Fields are float64 (or float32 bases under PR_MIXED) tensors of
n^3 contiguous values laid out [x][y][z]; a block of columns is a tensor of
shape (ncols, n^3).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import List, Optional, Sequence

from . import _lib as L
from ._lib import PR_F64, PR_MIXED, PR_FLOW_ABC, PR_FLOW_KOLMOGOROV, PR_FLOW_UNIFORM  # noqa: F401
from ._lib import PR_FLOW_ABC_T, PR_FLOW_KOLMOGOROV_T  # noqa: F401
from ._lib import PR_MODE_ADAPTIVE, PR_MODE_FIXED_POD, PR_MODE_COARSE_GRID  # noqa: F401

__all__ = ["Context", "PrError", "problem", "pr_fine_propagate", "pr_fine_tuned", "pr_gram", "pr_gram_noalloc", "pr_pod_build",
           "pr_coarse_propagate", "pr_parareal_solve", "pr_plan", "pr_footprint", "pr_solve_begin",
           "pr_solve_step_batch", "pr_solve_state", "pr_solve_done", "pr_solve_bytes", "pr_solve_end",
           "SolveHandle", "costmodel"]


class PrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{L.STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = L.STATUS.get(status, str(status))


def _torch():
    import torch
    return torch


def problem(n: int, kappa: float, flow: int, fp, precision: int = PR_F64,
            Lbox: float = 2 * math.pi) -> L.pr_grid_problem:
    p = L.pr_grid_problem()
    p.n = int(n)
    p.L = float(Lbox)
    p.kappa = float(kappa)
    p.flow = int(flow)
    for i in range(3):
        p.fp[i] = float(fp[i]) if i < len(fp) else 0.0
    p.precision = int(precision)
    return p


def problem_of(prob) -> L.pr_grid_problem:
    """From a workloads.Problem-like object (n, kappa, flow, fp, precision, L)."""
    return problem(prob.n, prob.kappa, prob.flow, prob.fp, getattr(prob, "precision", 0),
                   getattr(prob, "L", 2 * math.pi))


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_dev(t, dtype, numel=None, name="tensor"):
    torch = _torch()
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")


class Context:
    """pr_ctx on one HIP device (scratch memory, staging, velocity tables)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self.lib = L.load()
        h = ctypes.c_void_p()
        st = self.lib.pr_ctx_create(int(device), int(budget_bytes), ctypes.byref(h))
        if st != L.PR_OK:
            raise PrError(st, "pr_ctx_create failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.pr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def error(self) -> str:
        return self.lib.pr_last_error(self.h).decode()

    def check(self, st: int):
        if st != L.PR_OK:
            raise PrError(st, self.error())

    def scratch_bytes(self) -> int:
        return int(self.lib.pr_ctx_scratch_bytes(self.h))


def _fdtype(prob: L.pr_grid_problem):
    torch = _torch()
    return torch.float32 if prob.precision == PR_MIXED else torch.float64


def pr_fine_propagate(ctx: Context, items: Sequence[dict], stream=None):
    """items: dicts with prob, dt, n_steps, u_in, u_out and optional
    snap_every, snaps, t0 (see pr.h)."""
    torch = _torch()
    arr = (L.pr_fine_item * len(items))()
    keep = []
    for i, it in enumerate(items):
        prob = it["prob"]
        keep.append(prob)
        ng = prob.n ** 3
        _check_dev(it["u_in"], torch.float64, ng, "u_in")
        _check_dev(it["u_out"], torch.float64, ng, "u_out")
        arr[i].prob = ctypes.pointer(prob)
        arr[i].dt = float(it["dt"])
        arr[i].n_steps = int(it["n_steps"])
        arr[i].u_in = _ptr(it["u_in"])
        arr[i].u_out = _ptr(it["u_out"])
        se = int(it.get("snap_every", 0))
        arr[i].snap_every = se
        snaps = it.get("snaps")
        if snaps is not None:
            _check_dev(snaps, _fdtype(prob), ng * (int(it["n_steps"]) // se + 1), "snaps")
        arr[i].snaps = _ptr(snaps)
        arr[i].t0 = float(it.get("t0", 0.0))
    ctx.check(ctx.lib.pr_fine_propagate(ctx.h, len(items), arr, _stream(stream)))


def pr_fine_tuned(ctx: Context, precision: int, n: int, batch: int, planes: bool = False,
                  forced: bool = False, blocked: bool = False):
    """(tile_y, tile_z, threads[, x planes per workgroup][, blocked]) of the
    fused stencil launch shape chosen for a batch key (forced: the
    forced-flow stencil; blocked: 1 for a 2 x 2 register-blocked tiling), or
    None if no such batch ran yet."""
    ty, tz, nt, xp, bl = (ctypes.c_int() for _ in range(5))
    st = ctx.lib.pr_fine_tuned(ctx.h, int(precision), 1 if forced else 0, int(n), int(batch),
                               ctypes.byref(ty), ctypes.byref(tz), ctypes.byref(nt),
                               ctypes.byref(xp), ctypes.byref(bl))
    if st != L.PR_OK:
        return None
    out = (ty.value, tz.value, nt.value) + ((xp.value,) if planes else ())
    return out + ((bl.value,) if blocked else ())


def fine_kernel_name(ctx: Context, precision: int, n: int, batch: int) -> Optional[str]:
    """Name of the steady-flow stencil kernel and x chunk chosen for a batch
    key, as the profiler lists it (template arguments abbreviated)."""
    t = pr_fine_tuned(ctx, precision, n, batch, planes=True, blocked=True)
    if t is None:
        return None
    ty, tz, nt, xp, bl = t
    v = "double" if precision == L.PR_F64 else "float"
    return "%s<%s,%d,%d,%d>/x%d" % ("k_rk4_b22" if bl else "k_rk4_fused", v, ty, tz, nt, xp)


def pr_gram(ctx: Context, prob: L.pr_grid_problem, W, ncols: int, G_out=None, stream=None):
    """G = h^3 W^T W of a (ncols, N_g) column block; returns (ncols, ncols)."""
    torch = _torch()
    ng = prob.n ** 3
    _check_dev(W, _fdtype(prob), ncols * ng, "W")
    if G_out is None:
        G_out = torch.empty((ncols, ncols), dtype=torch.float64, device=W.device)
    _check_dev(G_out, torch.float64, ncols * ncols, "G_out")
    ctx.check(ctx.lib.pr_gram(ctx.h, ctypes.byref(prob), _ptr(W), int(ncols), _ptr(G_out),
                              _stream(stream)))
    return G_out


def pr_gram_noalloc(ctx: Context, prob: L.pr_grid_problem, W, G_out, stream=None, ncols=None):
    """pr_gram into a caller-provided (ncols, ncols) FP64 G_out, allocating
    nothing (the library's static device scratch)."""
    torch = _torch()
    ng = prob.n ** 3
    if ncols is None:
        ncols = G_out.shape[0]
    _check_dev(W, _fdtype(prob), ncols * ng, "W")
    _check_dev(G_out, torch.float64, ncols * ncols, "G_out")
    ctx.check(ctx.lib.pr_gram_noalloc(ctx.h, ctypes.byref(prob), _ptr(W), int(ncols),
                                      _ptr(G_out), _stream(stream)))
    return G_out


def pr_pod_build(ctx: Context, items: Sequence[dict], stream=None):
    """items: dicts with prob, blocks (list of (cols, N_g) tensors), gamma,
    cap, R_out ((cap, N_g) tensor), m_out (int32 device tensor) and optional
    block_valid (list of int32 device scalars or None), force_m,
    lambda_out."""
    torch = _torch()
    arr = (L.pr_pod_item * len(items))()
    keep = []
    for i, it in enumerate(items):
        prob = it["prob"]
        ng = prob.n ** 3
        blocks = it["blocks"]
        bp = (ctypes.c_void_p * len(blocks))()
        bc = (ctypes.c_int * len(blocks))()
        bv = (ctypes.c_void_p * len(blocks))()
        valid = it.get("block_valid") or [None] * len(blocks)
        for b, blk in enumerate(blocks):
            _check_dev(blk, _fdtype(prob), None, "block")
            if blk.numel() % ng:
                raise ValueError("block size must be a multiple of n^3")
            bp[b] = blk.data_ptr()
            bc[b] = blk.numel() // ng
            bv[b] = _ptr(valid[b])
        keep += [prob, bp, bc, bv]
        arr[i].prob = ctypes.pointer(prob)
        arr[i].n_blocks = len(blocks)
        arr[i].blocks = bp
        arr[i].block_cols = bc
        arr[i].block_valid = bv
        arr[i].gamma = float(it["gamma"])
        arr[i].cap = int(it["cap"])
        arr[i].force_m = int(it.get("force_m", -1))
        _check_dev(it["R_out"], _fdtype(prob), ng * int(it["cap"]), "R_out")
        _check_dev(it["m_out"], torch.int32, 1, "m_out")
        arr[i].R_out = _ptr(it["R_out"])
        arr[i].m_out = _ptr(it["m_out"])
        lo = it.get("lambda_out")
        if lo is not None:
            _check_dev(lo, torch.float64, sum(bc), "lambda_out")
        arr[i].lambda_out = _ptr(lo)
    ctx.check(ctx.lib.pr_pod_build(ctx.h, len(items), arr, _stream(stream)))


def pr_coarse_propagate(ctx: Context, items: Sequence[dict], stream=None):
    """items: dicts with prob, R ((cap, N_g) tensor), cap, m (int32 device
    scalar), u_in (list of 1 or 2 float64 fields), dT_total, and optional
    u_aug, n_c, dt_hint, u_out (list), beta_out, n_c_out, t0."""
    torch = _torch()
    arr = (L.pr_coarse_item * len(items))()
    keep = []
    for i, it in enumerate(items):
        prob = it["prob"]
        keep.append(prob)
        ng = prob.n ** 3
        cap = int(it["cap"])
        _check_dev(it["R"], _fdtype(prob), ng * cap, "R")
        _check_dev(it["m"], torch.int32, 1, "m")
        arr[i].prob = ctypes.pointer(prob)
        arr[i].R = _ptr(it["R"])
        arr[i].cap = cap
        arr[i].m = _ptr(it["m"])
        ua = it.get("u_aug")
        if ua is not None:
            _check_dev(ua, torch.float64, ng, "u_aug")
        arr[i].u_aug = _ptr(ua)
        ins = list(it["u_in"])
        arr[i].n_in = len(ins)
        for j, u in enumerate(ins):
            _check_dev(u, torch.float64, ng, "u_in")
            arr[i].u_in[j] = u.data_ptr()
        arr[i].dT_total = float(it["dT_total"])
        arr[i].n_c = int(it.get("n_c", 0))
        arr[i].dt_hint = float(it.get("dt_hint", 0.0))
        arr[i].t0 = float(it.get("t0", 0.0))
        outs = list(it.get("u_out") or [])
        for j, u in enumerate(outs):
            if u is not None:
                _check_dev(u, torch.float64, ng, "u_out")
            arr[i].u_out[j] = _ptr(u)
        bo = it.get("beta_out")
        if bo is not None:
            _check_dev(bo, torch.float64, len(ins) * (cap + 1), "beta_out")
        arr[i].beta_out = _ptr(bo)
        nco = it.get("n_c_out")
        if nco is not None:
            _check_dev(nco, torch.int32, 1, "n_c_out")
        arr[i].n_c_out = _ptr(nco)
    ctx.check(ctx.lib.pr_coarse_propagate(ctx.h, len(items), arr, _stream(stream)))


def opts_struct(o, U_ref=None) -> L.pr_parareal_opts:
    s = L.pr_parareal_opts()
    s.T = float(o.T)
    s.N = int(o.N)
    s.dt = float(o.dt)
    s.dM = int(getattr(o, "dM", 0))
    s.gamma1 = float(o.gamma1)
    s.gamma2 = float(o.gamma2)
    s.gamma3 = float(o.gamma3)
    s.cap0 = int(o.cap0)
    s.cap = int(o.cap)
    s.ml = int(o.ml)
    s.p = int(o.p)
    s.coarse_ratio = int(o.coarse_ratio)
    s.tol = float(o.tol)
    s.max_iter = int(getattr(o, "max_iter", 0))
    s.mode = int(getattr(o, "mode", 0))
    s.diag = int(getattr(o, "diag", 0))
    s.n_warm = int(getattr(o, "n_warm", 1))
    s.U_ref = _ptr(U_ref)
    return s


@dataclasses.dataclass
class Report:
    status: int
    iters: int
    converged: bool
    n_f: int
    dM: int
    n_s: int
    n_c: int
    n_sub: int
    m0: int
    jump: List[float]
    err: List[float]
    t_iter: List[float]
    ranks: List[List[int]]
    t_phase: dict
    fine_updates: float
    seconds: float
    # coarse-gap diagnostics (opts.diag): k -> values for n = k..N-2
    gap_fine: dict = dataclasses.field(default_factory=dict)
    gap_ref: dict = dataclasses.field(default_factory=dict)
    # max_ij |(Psi^T M Psi - I)_ij| of each recorded coarse step's basis
    basis_orth: dict = dataclasses.field(default_factory=dict)


class _ReportBuffers:
    """Host arrays a pr_report points into, sized for at most kmax iterations."""

    def __init__(self, N: int, max_iter: int, n_warm: int = 1):
        self.N = N
        self.Np = N - max(1, n_warm)          # parareal subintervals N'
        self.n_sub = max(self.Np, 1)
        kmax = max_iter if max_iter > 0 else self.Np
        kmax = max(0, min(kmax, self.Np))
        cap = kmax + 1
        self.jump = (ctypes.c_double * cap)()
        self.err = (ctypes.c_double * cap)()
        self.t_iter = (ctypes.c_double * cap)()
        self.ranks = (ctypes.c_int * (cap * self.n_sub))()
        self.gap_fine = (ctypes.c_double * (cap * self.n_sub))()
        self.gap_ref = (ctypes.c_double * (cap * self.n_sub))()
        self.basis_orth = (ctypes.c_double * (cap * self.n_sub))()
        self.rep = L.pr_report()
        self.rep.jump = self.jump
        self.rep.err = self.err
        self.rep.t_iter = self.t_iter
        self.rep.ranks = self.ranks
        self.rep.gap_fine = self.gap_fine
        self.rep.gap_ref = self.gap_ref
        self.rep.basis_orth = self.basis_orth

    def report(self, st: int, has_ref: bool) -> "Report":
        rep, k, n_sub, N = self.rep, self.rep.iters, self.n_sub, self.N
        return Report(status=st, iters=k, converged=bool(rep.converged), n_f=rep.n_f, dM=rep.dM,
                      n_s=rep.n_s, n_c=rep.n_c, n_sub=rep.n_sub, m0=rep.m0,
                      jump=[self.jump[i] for i in range(k)],
                      err=[self.err[i] for i in range(k + 1)] if has_ref else [],
                      t_iter=[self.t_iter[i] for i in range(k + 1)],
                      ranks=[[self.ranks[kk * n_sub + n] for n in range(kk, self.Np)]
                             for kk in range(1, k + 1)],
                      t_phase=dict(zip("FCUAG", list(rep.t_phase))),
                      fine_updates=rep.fine_updates, seconds=rep.seconds,
                      gap_fine=self._gaps(self.gap_fine, k), gap_ref=self._gaps(self.gap_ref, k),
                      basis_orth=self._gaps(self.basis_orth, k, keep_nan=True))

    def _gaps(self, arr, k, keep_nan=False):
        out = {}
        for kk in range(1, k + 1):
            row = [arr[kk * self.n_sub + n] for n in range(kk, self.Np)]
            if row and all(v >= 0 or (keep_nan and v != v) for v in row):
                out[kk] = row
        return out


def pr_parareal_solve(ctx: Context, prob: L.pr_grid_problem, opts, u0, U_out=None,
                      U_ref=None, stream=None, allow_notconv: bool = True):
    """Whole solve. Returns (U_out of shape (N + 1, N_g), Report)."""
    torch = _torch()
    ng = prob.n ** 3
    N = int(opts.N)
    _check_dev(u0, torch.float64, ng, "u0")
    if U_out is None:
        U_out = torch.empty((N + 1, ng), dtype=torch.float64, device=u0.device)
    _check_dev(U_out, torch.float64, (N + 1) * ng, "U_out")
    if U_ref is not None:
        _check_dev(U_ref, torch.float64, (N + 1) * ng, "U_ref")
    o = opts_struct(opts, U_ref)
    rb = _ReportBuffers(N, int(getattr(opts, "max_iter", 0)), int(getattr(opts, "n_warm", 1)))
    st = ctx.lib.pr_parareal_solve(ctx.h, ctypes.byref(prob), ctypes.byref(o), _ptr(u0),
                                   _ptr(U_out), ctypes.byref(rb.rep), _stream(stream))
    if st != L.PR_OK and not (allow_notconv and st == -5):
        raise PrError(st, ctx.error())
    return U_out, rb.report(st, U_ref is not None)


class SolveHandle:
    """An incremental solve (pr_solve_begin .. pr_solve_end). Keeps U_ref
    alive for the library, which reads it on every iteration."""

    def __init__(self, ctx: Context, h: int, prob, opts, U_ref):
        self.ctx = ctx
        self.h = h
        self.prob = prob
        self.opts = opts
        self.U_ref = U_ref

    @property
    def done(self) -> bool:
        return bool(self.ctx.lib.pr_solve_done(ctypes.c_void_p(self.h)))

    @property
    def nbytes(self) -> int:
        return int(self.ctx.lib.pr_solve_bytes(ctypes.c_void_p(self.h)))


def pr_solve_begin(ctx: Context, prob: L.pr_grid_problem, opts, u0, U_ref=None,
                   stream=None) -> SolveHandle:
    """Admit a solve and run its k = 0 step. Raises PrError (PR_ENOMEM when
    the context's budget cannot hold it)."""
    torch = _torch()
    ng = prob.n ** 3
    N = int(opts.N)
    _check_dev(u0, torch.float64, ng, "u0")
    if U_ref is not None:
        _check_dev(U_ref, torch.float64, (N + 1) * ng, "U_ref")
    o = opts_struct(opts, U_ref)
    out = ctypes.c_void_p()
    st = ctx.lib.pr_solve_begin(ctx.h, ctypes.byref(prob), ctypes.byref(o), _ptr(u0),
                                ctypes.byref(out), _stream(stream))
    if st != L.PR_OK:
        raise PrError(st, ctx.error())
    return SolveHandle(ctx, out.value, prob, opts, U_ref)


def pr_solve_step_batch(ctx: Context, handles, stream=None) -> List[bool]:
    """One parareal iteration of every unfinished handle; returns done flags."""
    n = len(handles)
    arr = (ctypes.c_void_p * max(n, 1))(*[h.h for h in handles])
    done = (ctypes.c_int * max(n, 1))()
    st = ctx.lib.pr_solve_step_batch(ctx.h, n, arr, done, _stream(stream))
    if st != L.PR_OK:
        raise PrError(st, ctx.error())
    return [bool(done[i]) for i in range(n)]


def pr_solve_state(ctx: Context, handle: SolveHandle, j: int, out=None, stream=None):
    """Copy of the latest iterate's state at t = j DeltaT (device tensor)."""
    torch = _torch()
    ng = handle.prob.n ** 3
    if out is None:
        out = torch.empty(ng, dtype=torch.float64, device="cuda")
    _check_dev(out, torch.float64, ng, "out")
    st = ctx.lib.pr_solve_state(ctx.h, ctypes.c_void_p(handle.h), int(j), _ptr(out),
                                _stream(stream))
    if st != L.PR_OK:
        raise PrError(st, ctx.error())
    return out


def pr_solve_done(handle: SolveHandle) -> bool:
    return handle.done


def pr_solve_bytes(handle: SolveHandle) -> int:
    return handle.nbytes


def pr_solve_end(ctx: Context, handle: SolveHandle, U_out=None, stream=None,
                 allow_notconv: bool = True):
    """Finish a handle: (U_out of shape (N + 1, N_g), Report); U_out=False
    copies nothing out (returns None). The handle is freed whatever the
    status."""
    torch = _torch()
    N = int(handle.opts.N)
    ng = handle.prob.n ** 3
    if U_out is None:
        U_out = torch.empty((N + 1, ng), dtype=torch.float64, device="cuda")
    if U_out is not False:
        _check_dev(U_out, torch.float64, (N + 1) * ng, "U_out")
    rb = _ReportBuffers(N, int(getattr(handle.opts, "max_iter", 0)),
                        int(getattr(handle.opts, "n_warm", 1)))
    h = handle.h
    handle.h = None
    st = ctx.lib.pr_solve_end(ctx.h, ctypes.c_void_p(h), None if U_out is False else _ptr(U_out),
                              ctypes.byref(rb.rep), _stream(stream))
    if st != L.PR_OK and not (allow_notconv and st == -5):
        raise PrError(st, ctx.error())
    return (None if U_out is False else U_out), rb.report(st, handle.U_ref is not None)


def pr_plan(prob: L.pr_grid_problem, opts) -> dict:
    """Derived sizes of a solve: n_sub, n_f, dt, dM, n_s, n_c, max_iter."""
    lib = L.load()
    o = opts_struct(opts)
    info = L.pr_plan_info()
    st = lib.pr_plan(ctypes.byref(prob), ctypes.byref(o), ctypes.byref(info))
    if st != L.PR_OK:
        raise PrError(st, "pr_plan failed")
    return {k: getattr(info, k) for k, _ in info._fields_}


def pr_footprint(prob: L.pr_grid_problem, opts) -> int:
    lib = L.load()
    o = opts_struct(opts)
    b = ctypes.c_size_t()
    st = lib.pr_footprint(ctypes.byref(prob), ctypes.byref(o), ctypes.byref(b))
    if st != L.PR_OK:
        raise PrError(st, "pr_footprint failed")
    return int(b.value)


from . import costmodel  # noqa: E402,F401
