"""Adaptive parareal iteration of the oracle (formula4, Algorithm 2).

Numbering (reading of where T_0 sits): [0, T] is split into N subintervals of
length DeltaT. The warm-up window [0, T_0] is the first w = opts.n_warm of
them (T_0 = w DeltaT; w = 1 in the paper's runs of the adaptive method, w = 2
for its Parareal-I runs, Sec. 4), so the parareal partition of [T_0, T] has
N' = N - w subintervals and states U_n at t_hat_n = (n + w) DeltaT,
n = 0..N'. U_0 is the fine solution at T_0 (u_hat_0 of Case I); the states
at DeltaT, ..., (w - 1) DeltaT inside the window are fine states too.

k = 0 (Algorithm 2, initialisation): fine solve on [0, T_0] with snapshots
(one sequence every dM steps over the whole window), POD_Mode(W, gamma_1)
gives G_0, and U^0_{n+1} = G_0(P U^0_n).

k >= 1 (Algorithm 2, the iteration):
  (i)   F(U^{k-1}_n) and the snapshots W^k_{n,0} for n = k-1..N'-1;
        POD_Mode(W^k_{n,0}, gamma_2) -> R^k_{n,0}.
  (ii)  W^k_n = [R_{n-m_l,0} .. R_{n,0} (latest iteration of each),
        R^{k-1}_{n,0} .. R^{k-p}_{n,0}]; blocks with index < 0 or iteration
        < 1 are omitted; POD_Mode(W^k_n, gamma_3) -> R^k_n.
  (iii) U^k_j = U^{k-1}_j for j < k and U^k_k = F(U^{k-1}_{k-1}): the two
        coarse terms cancel there because U^k_{k-1} = U^{k-1}_{k-1}.
  (iv)  sequentially for n = k..N'-1 (the sweep): augment R^k_n with U^k_n
        (eq12), then U^k_{n+1} = G(P U^k_n) + F(U^{k-1}_n) - G(P U^{k-1}_n).
  (v)   stopping ("while not converged" is unspecified): the jump
        e_k = max_{n>=1} ||U^k_n - U^{k-1}_n||_M / ||U^k_n||_M <= tol, or
        k = N' (finite termination, Sec. 2), or k = max_iter.

mode = 1 is the comparison method "Parareal-I" of Sec. 4: plain parareal
(formula4 without augmentation) whose coarse propagator is the Galerkin POD
propagator G_0 of the k = 0 step, kept for every iteration; steps (i) and
(ii) build no bases. Its POD window is the warm-up window [0, T_0] (the
paper takes T_0 = 2 DeltaT there: n_warm = 2).

mode = 2 is "Parareal-II" of Sec. 4: plain parareal whose coarse propagator
solves the same equation on the coarse n/2 grid (gridcoarse.py); no POD at
all. The warm-up subinterval and the numbering are kept, so all three modes
share U^0_0 = F(u0).

Coarse-gap diagnostics (Sec. 4, the dT = delta t experiments; opts.diag): at
iteration k >= 1 the sweep step from U_n to U_{n+1} (n = k..N'-1) records
  gap_fine = ||F(U^{k-1}_n) - G_k(P U^{k-1}_n)||_M / ||F(U^{k-1}_n)||_M,
  gap_ref  = ||U_{n+1} - G_k(P U^k_n)||_M / ||U_{n+1}||_M  (U_{n+1} the serial
             fine reference, when given),
with G_k the coarse propagator of that step (adaptive and fixed-POD modes).

Time: subinterval i of [0, T] starts at i DeltaT, so the warm-up solve starts
at t = 0 and the fine and coarse solves from U_n (n = 0..N'-1) start at
t_hat_n = (n + w) DeltaT; fine step j of a solve from t starts at t + j dt.
Only the forced time-dependent flows read the time.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import coarse as C
from . import fd
from . import gridcoarse as GC
from . import pod as P


@dataclasses.dataclass
class Result:
    U: List[np.ndarray]           # N + 1 states at t = j DeltaT (U[0] = u0)
    # (history[k][n] and ranks are in parareal numbering: time index n + w)
    iters: int
    converged: bool
    jumps: List[float]            # e_k, k = 1..iters
    errors: List[float]           # vs U_ref, k = 0..iters (empty without U_ref)
    ranks: Dict[int, List[int]]   # k -> [m^k_n for n = k..N'-1]
    ranks0: Dict[int, List[int]]  # k -> [m^k_{n,0} for n = k-1..N'-1]
    m0: int                       # rank of V^0_POD
    n_f: int
    dt: float
    dM: int
    n_c: int
    history: List[List[np.ndarray]]  # iterates per k (only with keep_history)
    t_phase: Dict[str, float]
    gap_fine: Dict[int, List[float]] = dataclasses.field(default_factory=dict)  # k -> n = k..N'-1
    gap_ref: Dict[int, List[float]] = dataclasses.field(default_factory=dict)


def _norm_m(x: np.ndarray, h3: float) -> float:
    return math.sqrt(h3 * float(np.vdot(x, x)))


def requested_dt(prob, opts) -> float:
    """opts.dt, or the automatic rule when it is <= 0."""
    return opts.dt if opts.dt > 0 else fd.auto_dt(prob)


def solve(prob, opts, u0: np.ndarray, U_ref: Optional[List[np.ndarray]] = None,
          tau_r: float = P.TAU_R_F64, keep_history: bool = False,
          trace: Optional[dict] = None) -> Result:
    """Algorithm 2 (see the module docstring). ``trace``, when a dict, receives
    the intermediate POD data of the adaptive mode for tests:
    trace[("R0", k, n)] = R^k_{n,0} (stage-1 basis of iteration k) and
    trace[("W", k, n)] = W^k_n (the stage-2 input of the sweep step from n)."""
    op = fd.Operator.of(prob)
    n = prob.n
    h3 = op.h ** 3
    N = opts.N
    dT_sub = opts.T / N
    n_f, dt = fd.steps_per_subinterval(dT_sub, requested_dt(prob, opts))
    dM = fd.snapshot_stride(n_f, opts.dM)
    nw = int(getattr(opts, "n_warm", 1))
    if not 1 <= nw <= N:
        raise ValueError("n_warm must be in [1, N]")
    Np = N - nw
    n_c0 = C.coarse_steps(n_f, opts.coarse_ratio)
    max_iter = opts.max_iter if opts.max_iter > 0 else Np
    t_phase = {"F": 0.0, "C": 0.0, "U": 0.0, "A": 0.0, "G": 0.0}
    u0v = np.asarray(u0, dtype=np.float64).reshape(-1)

    def t_hat(j):
        return (j + nw) * dT_sub

    def err_of(states):
        if U_ref is None:
            return None
        e = 0.0
        for j in range(1, len(states)):
            ref = np.asarray(U_ref[j + nw]).reshape(-1)
            e = max(e, _norm_m(states[j] - ref, h3) / _norm_m(ref, h3))
        return e

    # ---- k = 0: Case I ----------------------------------------------------
    t0 = time.perf_counter()
    ends, W = fd.fine_window(op, u0v.reshape(n, n, n), dt, n_f, nw, dM)
    t_phase["F"] += time.perf_counter() - t0
    U0hat = ends[-1].reshape(-1)
    warm = [u0v.copy()] + [e.reshape(-1) for e in ends[:-1]]   # time indices 0..w-1
    mode = getattr(opts, "mode", 0)
    if mode == 2:
        return _solve_coarse_grid(prob, opts, op, warm, U0hat, n_f, dt, dM, n_c0, max_iter,
                                  err_of, keep_history, t_phase, h3, nw)
    t0 = time.perf_counter()
    R0, m0, _ = P.pod_mode(W, opts.gamma1, h3, opts.cap, tau_r)
    t_phase["C"] += time.perf_counter() - t0
    del W
    t0 = time.perf_counter()
    sys0 = C.ReducedSystem(op, R0, h3)
    n_c = sys0.guarded_steps(dT_sub, n_c0)
    t_phase["U"] += time.perf_counter() - t0
    U_prev = [U0hat]
    t0 = time.perf_counter()
    for j in range(Np):
        beta = sys0.rk4(sys0.project(U_prev[-1]), t_hat(j), dT_sub, n_c)
        U_prev.append(R0 @ beta if m0 > 0 else np.zeros_like(U0hat))
    t_phase["G"] += time.perf_counter() - t0

    errors = []
    e0 = err_of(U_prev)
    if e0 is not None:
        errors.append(e0)
    history = [list(U_prev)] if keep_history else []

    hist: Dict[int, Dict[int, np.ndarray]] = {}
    jumps: List[float] = []
    ranks: Dict[int, List[int]] = {}
    ranks0: Dict[int, List[int]] = {}
    converged = Np == 0
    k = 0
    fixed = getattr(opts, "mode", 0) == 1
    diag = bool(getattr(opts, "diag", 0))
    gap_fine: Dict[int, List[float]] = {}
    gap_ref: Dict[int, List[float]] = {}

    def record_gaps(kk, nn, g_new, g_old):
        F = Fk[nn]
        gap_fine[kk].append(_norm_m(F - g_old, h3) / _norm_m(F, h3))
        if U_ref is not None:
            ref = np.asarray(U_ref[nn + 1 + nw]).reshape(-1)
            gap_ref[kk].append(_norm_m(ref - g_new, h3) / _norm_m(ref, h3))

    while not converged and k < max_iter:
        k += 1
        gap_fine[k] = []
        gap_ref[k] = []
        # (i) fine propagation and stage-1 POD, parallel over n
        Fk: Dict[int, np.ndarray] = {}
        hist[k] = {}
        ranks0[k] = []
        for nn in range(k - 1, Np):
            t0 = time.perf_counter()
            if fixed:
                Fn, _ = fd.fine_propagate(op, U_prev[nn].reshape(n, n, n), dt, n_f,
                                          t0=t_hat(nn))
            else:
                Fn, Wn = fd.fine_propagate(op, U_prev[nn].reshape(n, n, n), dt, n_f, dM,
                                           t0=t_hat(nn))
            t_phase["F"] += time.perf_counter() - t0
            Fk[nn] = Fn.reshape(-1)
            if fixed:
                continue
            t0 = time.perf_counter()
            R, m, _ = P.pod_mode(Wn, opts.gamma2, h3, opts.cap0, tau_r)
            t_phase["C"] += time.perf_counter() - t0
            hist[k][nn] = R
            ranks0[k].append(m)
            if trace is not None:
                trace[("R0", k, nn)] = R

        def latest(j):
            return hist[min(k, j + 1)][j]

        # (iii) converged prefix
        U_cur = [U_prev[j] for j in range(k)]
        U_cur.append(Fk[k - 1])
        ranks[k] = []
        # (ii) + (iv) sequential sweep
        for nn in range(k, Np):
            if fixed:
                # U^k_{n+1} = G_0(P U^k_n) + F(U^{k-1}_n) - G_0(P U^{k-1}_n)
                t0 = time.perf_counter()
                b_new = sys0.rk4(sys0.project(U_cur[nn]), t_hat(nn), dT_sub, n_c)
                b_old = sys0.rk4(sys0.project(U_prev[nn]), t_hat(nn), dT_sub, n_c)
                g_new = R0 @ b_new if m0 > 0 else np.zeros_like(Fk[nn])
                g_old = R0 @ b_old if m0 > 0 else np.zeros_like(Fk[nn])
                U_cur.append(g_new + Fk[nn] - g_old)
                t_phase["G"] += time.perf_counter() - t0
                if diag:
                    record_gaps(k, nn, g_new, g_old)
                continue
            t0 = time.perf_counter()
            blocks = [latest(j) for j in range(nn - opts.ml, nn + 1) if j >= 0]
            blocks += [hist[k - i][nn] for i in range(1, opts.p + 1) if k - i >= 1]
            Wkn = np.concatenate(blocks, axis=1)
            if trace is not None:
                trace[("W", k, nn)] = Wkn
            Rkn, mkn, _ = P.pod_mode(Wkn, opts.gamma3, h3, opts.cap, tau_r)
            t_phase["C"] += time.perf_counter() - t0
            ranks[k].append(mkn)
            t0 = time.perf_counter()
            Psi, _ = C.augment(Rkn, U_cur[nn], h3)
            t_phase["A"] += time.perf_counter() - t0
            t0 = time.perf_counter()
            sysr = C.ReducedSystem(op, Psi, h3)
            nc = sysr.guarded_steps(dT_sub, n_c0)
            t_phase["U"] += time.perf_counter() - t0
            t0 = time.perf_counter()
            b_new = sysr.rk4(sysr.project(U_cur[nn]), t_hat(nn), dT_sub, nc)
            b_old = sysr.rk4(sysr.project(U_prev[nn]), t_hat(nn), dT_sub, nc)
            g_new = Psi @ b_new if Psi.shape[1] else np.zeros_like(Fk[nn])
            g_old = Psi @ b_old if Psi.shape[1] else np.zeros_like(Fk[nn])
            U_cur.append(g_new + Fk[nn] - g_old)
            t_phase["G"] += time.perf_counter() - t0
            if diag:
                record_gaps(k, nn, g_new, g_old)
        # (v) jump
        e = 0.0
        for j in range(1, Np + 1):
            nrm = _norm_m(U_cur[j], h3)
            dj = _norm_m(U_cur[j] - U_prev[j], h3)
            e = max(e, dj / nrm if nrm > 0 else (0.0 if dj == 0 else math.inf))
        jumps.append(e)
        ek = err_of(U_cur)
        if ek is not None:
            errors.append(ek)
        if keep_history:
            history.append(list(U_cur))
        # drop bases no longer reachable: latest() needs hist[j+1][j] for
        # j < k - 1 and hist[k - i] for i <= p.
        for kk in list(hist.keys()):
            if kk < k - opts.p:
                keep = {j: v for j, v in hist[kk].items() if j == kk - 1}
                hist[kk] = keep
        U_prev = U_cur
        converged = (e <= opts.tol) or (k == Np)

    U_out = [u.copy() for u in warm] + [u.copy() for u in U_prev]
    return Result(U=U_out, iters=k, converged=converged, jumps=jumps, errors=errors,
                  ranks=ranks, ranks0=ranks0, m0=m0, n_f=n_f, dt=dt, dM=dM,
                  n_c=n_c, history=history, t_phase=t_phase,
                  gap_fine=gap_fine if diag else {}, gap_ref=gap_ref if diag else {})


def _solve_coarse_grid(prob, opts, op, warm, U0hat, n_f, dt, dM, n_c0, max_iter, err_of,
                       keep_history, t_phase, h3, nw) -> Result:
    """Parareal-II: U^0_{n+1} = G(U^0_n) and, for k >= 1,
    U^k_{n+1} = G(U^k_n) + F(U^{k-1}_n) - G(U^{k-1}_n), G the coarse-grid
    propagator (formula4 with the coarse spatial discretisation)."""
    n = prob.n
    N = opts.N
    Np = N - nw
    dT_sub = opts.T / N
    prob_c = GC.coarse_problem(prob)
    op_c = fd.Operator.of(prob_c)
    n_g = GC.grid_steps(prob_c, dT_sub, n_f, opts.coarse_ratio)

    def G(u, j):
        t0 = time.perf_counter()
        v = GC.coarse_grid_propagate(op_c, u, dT_sub, n_g, t0=(j + nw) * dT_sub)
        t_phase["G"] += time.perf_counter() - t0
        return v

    U_prev = [U0hat]
    for j in range(Np):
        U_prev.append(G(U_prev[-1], j))
    errors = []
    e0 = err_of(U_prev)
    if e0 is not None:
        errors.append(e0)
    history = [list(U_prev)] if keep_history else []
    jumps: List[float] = []
    converged = Np == 0
    k = 0
    while not converged and k < max_iter:
        k += 1
        Fk = {}
        for nn in range(k - 1, Np):
            t0 = time.perf_counter()
            Fn, _ = fd.fine_propagate(op, U_prev[nn].reshape(n, n, n), dt, n_f,
                                      t0=(nn + nw) * dT_sub)
            t_phase["F"] += time.perf_counter() - t0
            Fk[nn] = Fn.reshape(-1)
        U_cur = [U_prev[j] for j in range(k)]
        U_cur.append(Fk[k - 1])
        for nn in range(k, Np):
            U_cur.append(G(U_cur[nn], nn) + Fk[nn] - G(U_prev[nn], nn))
        e = 0.0
        for j in range(1, Np + 1):
            nrm = _norm_m(U_cur[j], h3)
            dj = _norm_m(U_cur[j] - U_prev[j], h3)
            e = max(e, dj / nrm if nrm > 0 else (0.0 if dj == 0 else math.inf))
        jumps.append(e)
        ek = err_of(U_cur)
        if ek is not None:
            errors.append(ek)
        if keep_history:
            history.append(list(U_cur))
        U_prev = U_cur
        converged = (e <= opts.tol) or (k == Np)
    U_out = [u.copy() for u in warm] + [u.copy() for u in U_prev]
    return Result(U=U_out, iters=k, converged=converged, jumps=jumps, errors=errors,
                  ranks={}, ranks0={}, m0=0, n_f=n_f, dt=dt, dM=dM, n_c=n_g,
                  history=history, t_phase=t_phase)


def reference(prob, opts, u0: np.ndarray) -> List[np.ndarray]:
    """Serial fine solution at t = j DeltaT, j = 0..N (eq. error's U_n)."""
    op = fd.Operator.of(prob)
    out = fd.serial_fine(op, np.asarray(u0, dtype=np.float64).reshape(prob.n, prob.n, prob.n),
                         opts.T / opts.N, opts.N, requested_dt(prob, opts))
    return [o.reshape(-1) for o in out]
