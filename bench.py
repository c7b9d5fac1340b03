"""Benchmark of the adaptive parareal hot path on one MI355X.

A step is one whole adaptive parareal solve (k = 0 initialisation, every
iteration's batched fine solves, both POD stages, the sequential
augmentation / coarse / correction sweep and the convergence check) of the
128^3 Kolmogorov FP64 workload (kappa = 0.01, T = 10 over 64 subintervals,
dt = 1e-3, POD rank <= 20), inputs resident in HBM.

Printed JSON line (rank 0, one line):
  value      fine grid-point RK4 updates per second of the whole solve (GPts/s)
  roofline   the fine-stencil stage kernel: algorithmic bytes per launch over
             its average launch duration (HIP events on the library's stream)
  cpu_baseline  the FP64 oracle's fine propagator on a bounded sample
plus the time to reach 1e-6 relative L2 against the serial fine solution.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FUSED_TILINGS = 11   # steady-flow stencil tilings (PR_FUSED_CFG indices)
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--stencil-only", action="store_true",
                    help="time only the batched fine propagator (profiling runs)")
    ap.add_argument("--stencil-f32", action="store_true",
                    help="with --stencil-only: the same fields with the FP32 stencil (PR_MIXED)")
    ap.add_argument("--no-ref", action="store_true",
                    help="skip the serial fine reference (no error history; profiling runs)")
    ap.add_argument("--sweep", action="store_true",
                    help="also time the fine step in every stencil tiling (stderr and JSON)")
    ap.add_argument("--gram-only", action="store_true",
                    help="time the snapshot Gram (pr_gram) of the 128^3 workload")
    ap.add_argument("--serve-study", action="store_true",
                    help="serving stream at scale: capacity, then Poisson phases at --serve-rates")
    ap.add_argument("--serve-rates", default="0.5,0.7,0.9")
    ap.add_argument("--serve-skip", type=int, default=8)
    ap.add_argument("--serve-capacity", type=float, default=0.0,
                    help="solves/s; 0 measures it with a closed loop first")
    ap.add_argument("--serve-requests", type=int, default=6,
                    help="requests per serving phase (closed loop, then Poisson); 0 = skip")
    ap.add_argument("--mixed256", action="store_true",
                    help="report run of the 256^3 ABC mixed-precision workload instead "
                         "(its own JSON line): error per iteration against the FP64 serial "
                         "fine solution")
    ap.add_argument("--ensemble", type=int, default=0,
                    help="report run of K ensemble instances solved together (own JSON line)")
    ap.add_argument("--max-iter", type=int, default=4,
                    help="iterations of the --mixed256 run")
    ap.add_argument("--study", action="store_true",
                    help="report run of the (m_l, p) x kappa grid on 32^3 ABC (own JSON line)")
    ap.add_argument("--paper-flow", action="store_true",
                    help="report run of the forced flows of Sec. 4 on 128^3 (own JSON line): "
                         "forced-stencil roofline and error per iteration of the three modes")
    ap.add_argument("--paper-N", type=int, default=41,
                    help="subintervals of the --paper-flow runs (DeltaT = 5)")
    ap.add_argument("--gap", action="store_true",
                    help="report run of the coarse-gap diagnostics (Sec. 4, dT = delta t) of the "
                         "adaptive method on the forced flows at 128^3 (own JSON line)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


CSRC = os.path.join(ROOT, "paper_2601_10981_amd", "csrc")
STENCIL_SRC = os.path.join(CSRC, "stencil.hip")
STENCIL_PROFILE = os.path.join(ROOT, "profiles", "k_rk4_fused_f64_kolmogorov128_batch63.md")
B22_SRC = os.path.join(CSRC, "stencil22.hip")
B22_PROFILE = os.path.join(ROOT, "profiles", "k_rk4_b22_f64_kolmogorov128_batch63.md")


def stencil_src_of(kname):
    return B22_SRC if kname.startswith("k_rk4_b22") else STENCIL_SRC


def stencil_profile_of(kname):
    return B22_PROFILE if kname.startswith("k_rk4_b22") else STENCIL_PROFILE


FORCED_SRC = os.path.join(CSRC, "forced.hip")
FORCED_PROFILE = os.path.join(ROOT, "profiles", "k_rk4_forced_f64_paperkolmogorov128_batch40.md")


def _sources_sha(paths):
    import hashlib
    h = hashlib.sha256()
    for q in paths:
        h.update(open(q, "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel, src=None, profile=STENCIL_PROFILE):
    """HBM bytes per launch of a stencil kernel from its committed PMC
    summary, or None when the kernel's sources (its .hip file and the shared
    stencil_dev.h) or its tiling changed since it was taken."""
    try:
        sha = _sources_sha([src or STENCIL_SRC, os.path.join(CSRC, "stencil_dev.h")])
        fields = {}
        for line in open(profile):
            if ":" in line and not line.startswith(("|", "#", " ")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        if fields.get("source_sha256_16") == sha and fields.get("kernel") == kernel:
            return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        pass
    return None


def _oracle_steps(args):
    """One worker of the CPU baseline: the oracle's RK4 steps on one field
    (subinterval i's copy of the workload's initial field) until the
    deadline; returns the steps taken."""
    wname, i, deadline = args
    import workloads as W
    from oracle import fd
    w = W.BY_NAME[wname]
    op = fd.Operator.of(w.problem)
    u = W.initial_field(w) * (1.0 + 0.01 * i)
    n_f, dt = fd.steps_per_subinterval(w.opts.T / w.opts.N, w.opts.dt)
    steps = 0
    while True:
        u = fd.rk4_step(op, u, dt)
        steps += 1
        if time.time() >= deadline:
            return steps


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s):
    """The oracle's fine propagator (numpy FP64, classical RK4) on the host's
    cores: one process per core, each stepping its own subinterval field of
    the workload (the batched fine solve's independent fields) until a common
    deadline; throughput = all steps x N_g / wall time. The core count is the
    host's usable CPU set, capped at 16 (the CPU share of one GPU here); each
    worker runs numpy single-threaded."""
    import multiprocessing as mp
    cores = min(16, len(os.sched_getaffinity(0)))
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_steps, [(w.name, i, time.time() + 0.5) for i in range(cores)])  # warm
        t0 = time.time()
        steps = pool.map(_oracle_steps, [(w.name, i, t0 + budget_s) for i in range(cores)])
        el = time.time() - t0
    ng = w.problem.n ** 3
    tot = sum(steps)
    return {"value": tot * ng / el / 1e9, "unit": "GPts/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{tot} RK4 steps on {cores} independent {w.problem.n}^3 fields of the "
                      f"workload, one process each (oracle fine propagator, numpy FP64, "
                      f"{el:.1f} s)"}


def copy_bandwidth(stream, nbytes=1 << 30, trials=3, back_to_back=10):
    """Achieved HBM bandwidth of plain device copies: torch's copy kernel and
    the HIP runtime's device-to-device copy, nbytes read and nbytes written
    per copy, back_to_back copies between two HIP events on the stream (so
    the events' own cost is spread over them); the best of trials, GB/s."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(trials):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(back_to_back):
            b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) * 1e-3 / back_to_back
        best = s if best is None else min(best, s)
    torch_gbs = round(2 * nbytes / best / 1e9, 1)
    # the runtime's own device-to-device copy (hipMemcpyAsync), from the HIP
    # runtime torch already loaded (same soname, so no second runtime)
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_int, ctypes.c_void_p]
    hip.hipMemcpyAsync.restype = ctypes.c_int
    d2d = 3   # hipMemcpyDeviceToDevice
    st = ctypes.c_void_p(stream.cuda_stream)
    best_rt = None
    for _ in range(trials):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(back_to_back):
            if hip.hipMemcpyAsync(b.data_ptr(), a.data_ptr(), nbytes, d2d, st) != 0:
                raise RuntimeError("hipMemcpyAsync failed")
        e1.record(stream)
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) * 1e-3 / back_to_back
        best_rt = s if best_rt is None else min(best_rt, s)
    del a, b
    return torch_gbs, round(2 * nbytes / best_rt / 1e9, 1)


def oracle_c1_phases():
    """The oracle's whole adaptive solve of the 32^3 ABC workload (T = 1 over
    8 subintervals) on one host core, with its per-phase times in the paper's
    breakdown (F, C, U, A, G) and its iteration count."""
    import workloads as W
    from oracle import parareal
    w = W.ABC_32_F64
    u0 = W.initial_field(w)
    t0 = time.perf_counter()
    r = parareal.solve(w.problem, w.opts, u0)
    el = time.perf_counter() - t0
    return {"workload": w.name, "seconds": round(el, 2), "iters": r.iters,
            "t_phase_s": {k: round(v, 3) for k, v in r.t_phase.items()},
            "gpts": round(r.iters and (sum((w.opts.N - 1 - k + 1) for k in range(1, r.iters + 1))
                                       + 1) * r.n_f * w.problem.n ** 3 / max(r.t_phase["F"], 1e-9)
                          / 1e9, 5)}


def serving_sample(pr, ctx, budget, k):
    """The serving stream: requests drawn as the ensemble (grid 64..256 in
    steps of 32, random flow, kappa, horizon, N; tolerance 1e-6; mixed
    precision). Phase 1 submits k requests at once (closed loop) to measure
    capacity; phase 2 feeds the next k as a Poisson stream at 0.7 x that
    capacity and reports arrival-to-result latency."""
    import workloads as W
    from paper_2601_10981_amd import serving
    ws = W.serving_requests(2 * k)

    def req(i, arrival):
        w = ws[i]
        return serving.Request(i, float(arrival), pr.problem_of(w.problem), w.opts,
                               lambda w=w: W.fourier_field_device(w.problem.n, w.seed,
                                                                  "cuda").reshape(-1))
    log(f"serving: closed loop, {k} requests")
    closed = serving.serve(ctx, [req(i, 0.0) for i in range(k)], budget)
    capacity = k / closed.wall
    rate = 0.7 * capacity
    arrivals = W.poisson_arrivals(k, rate, seed=5)
    log(f"serving: Poisson at {rate:.4f}/s, {k} requests")
    openl = serving.serve(ctx, [req(k + i, arrivals[i]) for i in range(k)], budget)
    lat = openl.latencies()
    P = serving.ServeStats.percentile
    return {"requests_per_phase": k, "closed_loop_solves_per_s": round(capacity, 4),
            "rate_per_s": round(rate, 4), "p50_latency_s": round(P(lat, 50), 3),
            "p99_latency_s": round(P(lat, 99), 3), "solves_per_s": round(k / openl.wall, 4),
            "mean_live": round(openl.mean_live, 2), "max_live": openl.max_live,
            "grids": [c.n for c in sorted(openl.completed, key=lambda c: c.rid)],
            "iters": [c.iters for c in sorted(openl.completed, key=lambda c: c.rid)],
            "sample": f"{k} closed-loop then {k} Poisson requests of the serving stream "
                      f"(seeds 5000..{5000 + 2 * k - 1}); no warm-up exclusion"}


def serving_study(args):
    """The serving stream at scale: a closed loop of K requests (all at
    t = 0) measures the capacity (solves/s), unless --serve-capacity gives
    it; then, for each load factor, K further requests arrive as a Poisson
    stream at that fraction of the capacity. Latency is arrival to result;
    the first --serve-skip requests of each phase are warm-up and left out
    of the percentiles. Every request has its own seed."""
    import torch
    import paper_2601_10981_amd as pr
    import workloads as W
    from paper_2601_10981_amd import serving
    k = args.serve_requests
    rates = [float(x) for x in args.serve_rates.split(",") if x]
    ws = W.serving_requests(k * (len(rates) + 1))
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.85 * free)
    ctx = pr.Context(0, budget_bytes=budget)

    def req(i, arrival):
        w = ws[i]
        return serving.Request(i, float(arrival), pr.problem_of(w.problem), w.opts,
                               lambda w=w: W.fourier_field_device(w.problem.n, w.seed,
                                                                  "cuda").reshape(-1))
    P = serving.ServeStats.percentile
    out = {"mode": "serving", "requests_per_phase": k, "skip": args.serve_skip,
           "budget_bytes": budget, "phases": []}

    def phase(name, st, offered):
        lat = st.latencies(skip=args.serve_skip)
        done = sorted(st.completed, key=lambda c: c.rid)
        out["phases"].append({
            "phase": name, "offered_per_s": offered, "n_latencies": len(lat),
            "p50_latency_s": round(P(lat, 50), 3), "p99_latency_s": round(P(lat, 99), 3),
            "mean_latency_s": round(sum(lat) / len(lat), 3),
            "solves_per_s": round(len(done) / st.wall, 4), "wall_s": round(st.wall, 1),
            "mean_live": round(st.mean_live, 2), "max_live": st.max_live,
            "iters_mean": round(sum(c.iters for c in done) / len(done), 1),
            "not_converged": sum(1 for c in done if c.status != 0)})
        log(f"serving {name}: {out['phases'][-1]}")

    if args.serve_capacity > 0:
        capacity = args.serve_capacity
        out["capacity_given"] = capacity
    else:
        log(f"serving: closed loop, {k} requests")
        closed = serving.serve(ctx, [req(i, 0.0) for i in range(k)], budget,
                               log=lambda m: log("  " + m))
        capacity = k / closed.wall
        phase("closed_loop", closed, None)
    out["closed_loop_solves_per_s"] = round(capacity, 4)
    for j, f in enumerate(rates):
        rate = f * capacity
        arrivals = W.poisson_arrivals(k, rate, seed=5 + j)
        base = k * (j + 1)
        log(f"serving: Poisson at {f} x capacity = {rate:.4f}/s, {k} requests")
        st = serving.serve(ctx, [req(base + i, arrivals[i]) for i in range(k)], budget,
                           log=lambda m: log("  " + m))
        phase(f"poisson_{f}", st, round(rate, 4))
    out["sample"] = (f"{k} requests per phase (seeds 5000..{5000 + len(ws) - 1}), the first "
                     f"{args.serve_skip} of each phase excluded from the percentiles")
    ctx.close()
    print(json.dumps(out))


def gram_run(args):
    """The snapshot Gram G = h^3 W^T W (Algorithm 1, step 1) of the 128^3
    workload through pr_gram: a stage-1 block of n_s = 16 snapshot columns
    and a stage-2 collection of 48 columns, FP64 (FP64 MFMA) and FP32 data
    (FP32 MFMA products, FP64 sums). Reports the time per call (HIP events
    on the stream the library launches on), the algorithmic bytes (every
    column read once) and flops (2 N_g per entry of the upper block
    triangle of 16 x 16 tiles the kernel forms)."""
    import torch
    import paper_2601_10981_amd as pr
    import workloads as W
    n = 128
    ng = n ** 3
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = pr.Context(0)
    out = {"mode": "gram", "n": n, "cases": []}
    for prec, dt, vb in ((W.PREC_F64, torch.float64, 8), (W.PREC_MIXED, torch.float32, 4)):
        prob = pr.problem_of(W.Problem(n=n, kappa=0.01, flow=W.FLOW_KOLMOGOROV, fp=(1.0, 4.0, 0.0),
                                       precision=prec))
        for ncols in (16, 48):
            Wt = torch.randn((ncols, ng), dtype=torch.float64, device="cuda").to(dt)
            G = torch.empty((ncols, ncols), dtype=torch.float64, device="cuda")
            for _ in range(3):
                pr.pr_gram(ctx, prob, Wt, ncols, G)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record(stream)
            for _ in range(reps):
                pr.pr_gram(ctx, prob, Wt, ncols, G)
            e1.record(stream)
            torch.cuda.synchronize()
            s = e0.elapsed_time(e1) * 1e-3 / reps
            na = (ncols + 15) // 16
            flops = 2.0 * (na * (na + 1) // 2) * 256 * ng
            bytes_ = ncols * ng * vb
            out["cases"].append({"precision": "f64" if vb == 8 else "f32 data", "ncols": ncols,
                                 "us_per_call": round(s * 1e6, 1),
                                 "gb_s": round(bytes_ / s / 1e9, 1),
                                 "tflop_s": round(flops / s / 1e12, 2),
                                 "flop_per_byte": round(flops / bytes_, 2)})
            log(f"gram {out['cases'][-1]}")
            del Wt
    ctx.close()
    print(json.dumps(out))


def paper_projection(rep, serial_s, N):
    """The paper's speedup estimate T_F N / (T_total (k + 1)) with
    T_total = T_F + T_U + T_C + N (T_G + T_A) (Sec. 4), each term per
    subinterval as one processor group per subinterval would see it: T_F the
    serial fine time of one subinterval on this GPU, T_C and T_U the batched
    POD and reduced-operator times divided by the subintervals they served,
    T_A and T_G the sweep's augmentation and coarse times per coarse step."""
    from paper_2601_10981_amd import costmodel
    if serial_s is None or rep.iters < 1:
        return None
    Np, K = N - 1, rep.iters
    sweep = sum(Np - k for k in range(1, K + 1)) + Np        # + the k = 0 sweep
    pod = sum((Np - k + 1) + (Np - k) for k in range(1, K + 1)) + 1
    T_F = serial_s / N
    T_C = rep.t_phase["C"] / pod
    T_U = rep.t_phase["U"] / sweep
    T_A = rep.t_phase["A"] / sweep
    T_G = rep.t_phase["G"] / sweep
    T_total = costmodel.t_total(T_F, T_U, T_C, T_G, T_A, N)
    return {"T_F_s": round(T_F, 6), "T_C_s": round(T_C, 6), "T_U_s": round(T_U, 6),
            "T_A_s": round(T_A, 6), "T_G_s": round(T_G, 6), "T_total_s": round(T_total, 6),
            "k": K, "speedup_estimate": round(costmodel.speedup_estimate(T_F, T_total, N, K), 4),
            "note": "one processor group per subinterval, as the paper's estimate assumes; "
                    "phase times from a solve with one stream"}


def mixed256_run(args):
    """256^3 ABC, kappa = 0.005, T = 50 over 128 subintervals, dt = 5e-4: the
    stencil and the snapshot Grams in FP32, the rest in FP64. The FP64
    serial fine solution (computed on the GPU with the FP64 stencil first)
    is the reference of the per-iteration error."""
    import dataclasses
    import torch
    import paper_2601_10981_amd as pr
    import workloads as W
    w = W.ABC_256_MIXED
    n, N = w.problem.n, w.opts.N
    ng = n ** 3
    opts = dataclasses.replace(w.opts, max_iter=args.max_iter)
    p32 = pr.problem_of(w.problem)
    p64 = pr.problem_of(dataclasses.replace(w.problem, precision=W.PREC_F64))
    plan = pr.pr_plan(p32, opts)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    U_ref = torch.empty((N + 1, ng), dtype=torch.float64, device="cuda")
    U_out = torch.empty_like(U_ref)
    U_ref[0].copy_(W.fourier_field_device(n, w.seed, "cuda").reshape(-1))
    free, _ = torch.cuda.mem_get_info()
    ctx = pr.Context(0, budget_bytes=int(0.92 * free))
    log(f"mixed256: FP64 serial reference, {N} x {plan['n_f']} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(N):
        pr.pr_fine_propagate(ctx, [dict(prob=p64, dt=plan["dt"], n_steps=plan["n_f"],
                                        u_in=U_ref[j], u_out=U_ref[j + 1])])
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - t0
    log(f"mixed256: solve, max_iter {opts.max_iter}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the incremental form of the solve (bitwise the same iterates as
    # pr_parareal_solve), so that every iteration reports progress
    h = pr.pr_solve_begin(ctx, p32, opts, U_ref[0], U_ref=U_ref)
    k = 0
    t_diag = 0.0      # progress checks, excluded from the solve time
    state = torch.empty(ng, dtype=torch.float64, device="cuda")
    while not pr.pr_solve_done(h):
        pr.pr_solve_step_batch(ctx, [h])
        k += 1
        msg = f"  iteration {k} done at {time.perf_counter() - t0 - t_diag:.1f} s"
        if k <= 4 or k % 16 == 0:
            td = time.perf_counter()
            e = 0.0
            for j in range(1, N + 1):
                pr.pr_solve_state(ctx, h, j, out=state)
                e = max(e, (torch.linalg.vector_norm(state - U_ref[j]) /
                            torch.linalg.vector_norm(U_ref[j])).item())
            msg += f", max rel error {e:.3e}"
            t_diag += time.perf_counter() - td
        log(msg)
    _, rep = pr.pr_solve_end(ctx, h, U_out=U_out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0 - t_diag
    # the converged prefix U_j, j <= k + 1, is the FP32-stencil serial fine
    # solution: its distance to the FP64 one is the mixed-precision error of F
    prefix = [float("%.3e" % (torch.linalg.vector_norm(U_out[j] - U_ref[j]) /
                              torch.linalg.vector_norm(U_ref[j])).item())
              for j in range(1, rep.iters + 2)]
    out = {"mode": "mixed256", "workload": w.name, "n": n, "N": N, "n_f": plan["n_f"],
           "dt": plan["dt"], "cap0": opts.cap0, "cap": opts.cap, "precision": "mixed",
           "dtype": "f32 stencil and snapshot Gram; f64 eigen, re-orthogonalisation, sweep",
           "iters": rep.iters, "status": rep.status, "m0": rep.m0,
           "err_vs_fp64_serial": [float("%.3e" % e) for e in rep.err],
           "jump": [float("%.3e" % e) for e in rep.jump],
           "t_iter_s": [round(t, 2) for t in rep.t_iter],
           "t_phase_s": {k: round(v, 3) for k, v in rep.t_phase.items()},
           "solve_s": round(el, 2), "fine_updates": rep.fine_updates,
           "gpts_whole_solve": round(rep.fine_updates / el / 1e9, 2),
           "serial_fp64_s": round(serial_s, 2),
           "serial_fp64_gpts": round(N * plan["n_f"] * ng / serial_s / 1e9, 2),
           "fine_gpts_in_solve": round(rep.fine_updates / max(rep.t_phase["F"], 1e-9) / 1e9, 1),
           "prefix_err_vs_fp64": prefix,
           "ranks_last": rep.ranks[-1] if rep.ranks else None}
    ctx.close()
    print(json.dumps(out))


def ensemble_run(args):
    """K independent instances of the ensemble (grids 64..192, ABC or
    Kolmogorov, random kappa, T, N; mixed precision; tol 1e-6) admitted at
    once and advanced together: every step batches the fine solves and
    per-subinterval POD of all live instances into shared launches."""
    import torch
    import paper_2601_10981_amd as pr
    import workloads as W
    from paper_2601_10981_amd import serving
    ws = W.ensemble(args.ensemble)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.85 * free)
    ctx = pr.Context(0, budget_bytes=budget)
    reqs = [serving.Request(i, 0.0, pr.problem_of(w.problem), w.opts,
                            lambda w=w: W.fourier_field_device(w.problem.n, w.seed,
                                                               "cuda").reshape(-1))
            for i, w in enumerate(ws)]
    log(f"ensemble: {len(reqs)} instances")
    st = serving.serve(ctx, reqs, budget, max_live=len(reqs),
                       log=lambda m: log("  " + m))
    done = sorted(st.completed, key=lambda c: c.rid)
    # each instance's state at T against its own serial fine solution with
    # the FP64 stencil (after the timed loop)
    log("ensemble: FP64 serial references")
    errs, errs0 = [], []
    for r, w in zip(reqs, ws):
        import dataclasses
        p64 = pr.problem_of(dataclasses.replace(w.problem, precision=W.PREC_F64))
        plan = pr.pr_plan(p64, w.opts)
        u = W.fourier_field_device(w.problem.n, w.seed, "cuda").reshape(-1).clone()
        n0 = torch.linalg.vector_norm(u).item()
        v = torch.empty_like(u)
        for j in range(w.opts.N):
            pr.pr_fine_propagate(ctx, [dict(prob=p64, dt=plan["dt"], n_steps=plan["n_f"],
                                            u_in=u, u_out=v, t0=j * w.opts.T / w.opts.N)])
            u, v = v, u
        torch.cuda.synchronize()
        d = torch.linalg.vector_norm(r.result - u).item()
        errs.append(d / torch.linalg.vector_norm(u).item())
        errs0.append(d / n0)
    out = {"mode": "ensemble", "instances": len(done), "wall_s": round(st.wall, 2),
           "solves_per_s": round(len(done) / st.wall, 4), "steps": st.steps,
           "fine_gpts": round(sum(c.fine_updates for c in done) / st.wall / 1e9, 1),
           "mean_live": round(st.mean_live, 2), "max_live": st.max_live,
           "grids": [c.n for c in done], "N": [c.N for c in done],
           "iters": [c.iters for c in done], "status": [c.status for c in done],
           "err_at_T_vs_fp64_serial": [float("%.2e" % e) for e in errs],
           "max_err_at_T": float("%.3e" % max(errs)),
           # the same difference relative to the initial field: the FP32
           # stencil's rounding floor does not decay with the solution
           "err_at_T_rel_initial": [float("%.2e" % e) for e in errs0],
           "max_err_at_T_rel_initial": float("%.3e" % max(errs0)),
           "decay_at_T": [float("%.2e" % (a / b)) if b > 0 else None
                          for a, b in zip(errs0, errs)],
           "seeds": f"4000..{4000 + len(done) - 1}"}
    ctx.close()
    print(json.dumps(out))


def study_run(args):
    """The paper's experimental grid on this discretisation: every local
    collection (m_l, p) in {0,1}^2, and the fixed-POD and coarse-grid
    comparison methods, against the diffusivity, on 32^3 ABC
    (A = B = C = 1) with the blob initial field of seed 1, T = 2 over 16
    subintervals, dt = 2e-3, caps 10/10, tol 1e-8. Reports iterations to
    tol, the first iteration at or below 1e-6 relative L2 error against the
    serial fine solution, and the solve time."""
    import torch
    import paper_2601_10981_amd as pr
    import workloads as W
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = pr.Context(0)
    n, N = 32, 16
    u0 = torch.from_numpy(W.blob_field(n, 1).reshape(-1).copy()).cuda()
    rows = []
    for kappa in (0.5, 0.1, 0.05, 0.01):
        prob = pr.problem_of(W.Problem(n=n, kappa=kappa, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0)))
        base = W.PararealOpts(T=2.0, N=N, dt=2e-3, cap0=10, cap=10, tol=1e-8)
        plan = pr.pr_plan(prob, base)
        ref = torch.empty((N + 1, n ** 3), dtype=torch.float64, device="cuda")
        ref[0].copy_(u0)
        for j in range(N):
            pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=plan["dt"], n_steps=plan["n_f"],
                                            u_in=ref[j], u_out=ref[j + 1])])
        for ml, p, mode in ((0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (0, 0, 2)):
            # Parareal-I builds its fixed POD basis over T_0 = 2 DeltaT (Sec. 4)
            opts = W.PararealOpts(**{**base.__dict__, "ml": ml, "p": p, "mode": mode,
                                     "n_warm": 2 if mode == W.MODE_FIXED_POD else 1})
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rep = pr.pr_parareal_solve(ctx, prob, opts, u0, U_ref=ref)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            k6 = next((k for k, e in enumerate(rep.err) if e <= 1e-6), None)
            rows.append({"kappa": kappa,
                         "method": ("adaptive", "fixed-POD", "coarse-grid")[mode],
                         "ml": ml, "p": p, "iters": rep.iters, "m0": rep.m0,
                         "k_err_1e-6": k6, "err_final": float("%.3e" % rep.err[-1]),
                         "err_k1_k3": [float("%.2e" % e) for e in rep.err[1:4]],
                         "solve_s": round(el, 3)})
            log(f"study kappa={kappa} mode={mode} (m_l,p)=({ml},{p}): iters {rep.iters}, "
                f"k(1e-6) {k6}")
    ctx.close()
    print(json.dumps({"mode": "study", "n": n, "N": N, "T": 2.0, "flow": "ABC", "rows": rows}))


def paper_flow_run(args):
    """The forced flows of Sec. 4 (the Kolmogorov flow of eq. koleq and the
    ABC flow with phase sin(t)) at the paper's 2,097,152 unknowns (128^3) and
    its time parameters: delta t = 1e-2, DeltaT = 5 (n_f = 500), coarse step
    dT = 0.5 (coarse_ratio 50), the paper's gamma_1..3, initial value h = 0.
    delta_M = 10 (the paper's 5 would give 101 snapshots per subinterval, above
    the 64-column POD input), epsilon = 0.01 (one of the paper's AdapParareal
    cases; its explicit RK4 step is stable at delta t = 1e-2), N = --paper-N
    subintervals (the paper: 201), rank caps 21 / 31. For each flow: the
    forced stencil's roofline on the batched fine launch of one iteration,
    then the adaptive method ((m_l, p) = (1, 1)) and the two comparison
    methods, error per iteration against the serial fine solution."""
    import dataclasses
    import torch
    import paper_2601_10981_amd as pr
    import workloads as W
    n, N, dt, dTs = 128, args.paper_N, 1e-2, 5.0
    ng = n ** 3
    base = W.PararealOpts(T=dTs * N, N=N, dt=dt, dM=10, gamma1=1.0 - 5.0e-6,
                          gamma2=1.0 - 5.0e-6, gamma3=1.0 - 2.0e-8, cap0=21, cap=31, ml=1, p=1,
                          coarse_ratio=50, tol=1e-6, max_iter=args.max_iter)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    free, _ = torch.cuda.mem_get_info()
    ctx = pr.Context(0, budget_bytes=int(0.85 * free))
    out = {"metric": "forced flows of Sec. 4: forced-stencil GPts/s + %HBM; error per iteration",
           "n": n, "dofs": ng, "dt": dt, "DeltaT": dTs, "N": N, "T": dTs * N, "kappa": 0.01,
           "dM": base.dM, "coarse_ratio": base.coarse_ratio, "cap0": base.cap0, "cap": base.cap,
           "initial_value": "h = 0 (Sec. 4)", "flows": {}}
    for name, flow in (("kolmogorov", W.FLOW_KOLMOGOROV_T), ("abc", W.FLOW_ABC_T)):
        prob = pr.problem(n, 0.01, flow, (1.0, 1.0, 1.0))
        plan = pr.pr_plan(prob, base)
        n_f = plan["n_f"]
        res = {"n_f": n_f, "n_c": plan["n_c"]}
        # forced-stencil roofline: the batched fine launch of one iteration
        B = N - 1
        log(f"paper flow {name}: stencil timing {B} x {n}^3, {n_f} steps")
        xin = torch.stack([W.fourier_field_device(n, 11 + i, "cuda").reshape(-1) for i in range(B)])
        xout = torch.empty_like(xin)
        items = [dict(prob=prob, dt=plan["dt"], n_steps=n_f, u_in=xin[i], u_out=xout[i],
                      t0=(i + 1) * dTs) for i in range(B)]
        pr.pr_fine_propagate(ctx, items)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pr.pr_fine_propagate(ctx, items)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        avg = ms * 1e-3 / n_f
        bpl = 16 * ng * B
        tiling = pr.pr_fine_tuned(ctx, pr.PR_F64, n, B, planes=True, forced=True)
        kname = ("k_rk4_forced<double,%d,%d,%d>/x%d" % tiling) if tiling else "k_rk4_forced<double>"
        achieved = bpl / avg / 1e9
        res["stencil_gpts"] = round(B * ng * n_f / (ms * 1e-3) / 1e9, 2)
        res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": profiled_traffic(kname, FORCED_SRC, FORCED_PROFILE)
                           if name == "kolmogorov" else None,
                           "kernel": kname, "avg_launch_us": round(avg * 1e6, 2),
                           "bytes_per_launch": bpl}
        log(f"  {res['stencil_gpts']} GPts/s, {res['roofline']['frac']} of HBM peak")
        if args.sweep:
            sweep = {}
            for pol in range(3):
                os.environ["PR_FUSED_CHUNK"] = str(pol)
                for cfg in range(5):
                    os.environ["PR_FORCED_CFG"] = str(cfg)
                    pr.pr_fine_propagate(ctx, items)
                    e0.record(stream)
                    pr.pr_fine_propagate(ctx, items)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    t = pr.pr_fine_tuned(ctx, pr.PR_F64, n, B, forced=True)
                    key = "%dx%dx%d/chunks%d" % (t + (pol,))
                    sweep[key] = round(B * ng * n_f / (e0.elapsed_time(e1) * 1e-3) / 1e9, 2)
                    log(f"  tiling {key}: {sweep[key]} GPts/s")
            del os.environ["PR_FORCED_CFG"]
            del os.environ["PR_FUSED_CHUNK"]
            res["roofline"]["sweep_gpts"] = sweep
        del xin, xout
        if args.stencil_only:
            out["flows"][name] = res
            break
        # serial fine reference from h = 0
        U_ref = torch.zeros((N + 1, ng), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(N):
            pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=plan["dt"], n_steps=n_f, u_in=U_ref[j],
                                            u_out=U_ref[j + 1], t0=j * dTs)])
        torch.cuda.synchronize()
        res["serial_fine_s"] = round(time.perf_counter() - t0, 3)
        u0 = torch.zeros(ng, dtype=torch.float64, device="cuda")
        for mname, mode in (("adaptive_ml1_p1", W.MODE_ADAPTIVE), ("parareal_I_fixed_pod",
                                                                   W.MODE_FIXED_POD),
                            ("parareal_II_coarse_grid", W.MODE_COARSE_GRID)):
            opts = dataclasses.replace(base, mode=mode)
            if mode == W.MODE_FIXED_POD:
                # Parareal-I: the fixed basis from T_0 = 2 DeltaT = 10 (Sec. 4);
                # delta_M = 20 keeps its 1000 warm-up steps within 64 snapshots
                opts = dataclasses.replace(opts, n_warm=2, dM=20)
            log(f"  {mname}")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                _, rep = pr.pr_parareal_solve(ctx, prob, opts, u0, U_ref=U_ref)
            except pr.PrError as e:
                res[mname] = {"error": e.name}
                continue
            el = time.perf_counter() - t0
            res[mname] = {"iters": rep.iters, "converged": rep.converged, "seconds": round(el, 3),
                          "m0": rep.m0, "err_history": [float("%.3e" % e) for e in rep.err],
                          "jump_history": [float("%.3e" % e) for e in rep.jump],
                          "t_iter_s": [round(t, 3) for t in rep.t_iter],
                          "t_phase_s": {k: round(v, 3) for k, v in rep.t_phase.items()},
                          "ranks_k1": rep.ranks[0][:8] if rep.ranks else None}
            log(f"    iters {rep.iters} err {res[mname]['err_history']}")
        out["flows"][name] = res
        del U_ref
        torch.cuda.empty_cache()
    if args.stencil_only:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = a.numel() * 8
    ctx.close()
    print(json.dumps(out))


def gap_run(args):
    """The paper's dT = delta t experiments (Sec. 4): the coarse step equals
    the fine one, so the coarse propagator differs from the fine one only by
    the POD reduction in space. For both forced flows at 128^3 and epsilon in
    {0.05, 0.01, 0.005} the adaptive method ((m_l, p) = (1, 1)) records per
    iteration k and subinterval n the gaps
      ||F(U^{k-1}_n) - G_k(U^{k-1}_n)|| / ||F(U^{k-1}_n)|| and
      ||U_{n+1} - G_k(U^k_n)|| / ||U_{n+1}||.
    delta t = 1e-2 (epsilon = 0.05: 5e-3, the explicit RK4 bound), DeltaT = 5,
    delta_M = 10, h = 0, caps 21 / 31, N = --paper-N // 2 subintervals."""
    import dataclasses
    import statistics
    import torch
    import paper_2601_10981_amd as pr
    import workloads as W
    n, dTs = 128, 5.0
    N = max(3, args.paper_N // 2)
    ng = n ** 3
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    free, _ = torch.cuda.mem_get_info()
    ctx = pr.Context(0, budget_bytes=int(0.85 * free))
    out = {"metric": "coarse-gap diagnostics of the adaptive method, dT = delta t (Sec. 4)",
           "n": n, "N": N, "DeltaT": dTs, "max_iter": args.max_iter, "runs": []}
    for name, flow in (("kolmogorov", W.FLOW_KOLMOGOROV_T), ("abc", W.FLOW_ABC_T)):
        for eps in (0.05, 0.01, 0.005):
            dt = 1e-2 if eps < 0.05 else 5e-3
            n_f = int(round(dTs / dt))
            opts = W.PararealOpts(T=dTs * N, N=N, dt=dt, dM=n_f // 50, cap0=21, cap=31, ml=1, p=1,
                                  coarse_ratio=1, tol=1e-10, max_iter=args.max_iter, diag=1)
            prob = pr.problem(n, eps, flow, (1.0, 1.0, 1.0))
            U_ref = torch.zeros((N + 1, ng), dtype=torch.float64, device="cuda")
            for j in range(N):
                pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=n_f, u_in=U_ref[j],
                                                u_out=U_ref[j + 1], t0=j * dTs)])
            u0 = torch.zeros(ng, dtype=torch.float64, device="cuda")
            log(f"gap run {name} eps={eps}")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rep = pr.pr_parareal_solve(ctx, prob, opts, u0, U_ref=U_ref)
            el = time.perf_counter() - t0
            row = {"flow": name, "eps": eps, "dt": dt, "iters": rep.iters, "seconds": round(el, 2),
                   "err_history": [float("%.3e" % e) for e in rep.err], "gap_fine": {}, "gap_ref": {}}
            for key, src in (("gap_fine", rep.gap_fine), ("gap_ref", rep.gap_ref)):
                for k, vals in src.items():
                    row[key][k] = {"max": float("%.3e" % max(vals)),
                                   "median": float("%.3e" % statistics.median(vals))}
            log(f"  iters {rep.iters}; max fine gap per k "
                f"{[row['gap_fine'][k]['max'] for k in sorted(row['gap_fine'])]}")
            out["runs"].append(row)
            del U_ref
            torch.cuda.empty_cache()
    ctx.close()
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.mixed256:
        return mixed256_run(args)
    if args.ensemble > 0:
        return ensemble_run(args)
    if args.study:
        return study_run(args)
    if args.paper_flow:
        return paper_flow_run(args)
    if args.gap:
        return gap_run(args)
    if args.serve_study:
        return serving_study(args)
    if args.gram_only:
        return gram_run(args)
    import numpy as np
    import torch
    import paper_2601_10981_amd as pr
    import workloads as W

    import dataclasses
    w = W.KOL_128_F64
    f32 = args.stencil_only and args.stencil_f32
    prec = pr.PR_MIXED if f32 else pr.PR_F64
    prob = pr.problem_of(dataclasses.replace(w.problem, precision=W.PREC_MIXED) if f32
                         else w.problem)
    opts = w.opts
    n = w.problem.n
    ng = n ** 3
    N = opts.N
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.85 * free)
    ctx = pr.Context(0, budget_bytes=budget)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    u0 = torch.from_numpy(W.initial_field(w).reshape(-1).copy()).cuda()

    plan = pr.pr_plan(prob, opts)
    n_f, dt = plan["n_f"], plan["dt"]

    U_ref = None
    serial_s = None
    if not args.stencil_only and not args.no_ref:
        # serial fine reference (outside the timed region)
        log("serial fine reference")
        U_ref = torch.empty((N + 1, ng), dtype=torch.float64, device="cuda")
        U_ref[0].copy_(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(N):
            pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=n_f, u_in=U_ref[j],
                                            u_out=U_ref[j + 1])])
        torch.cuda.synchronize()
        serial_s = time.perf_counter() - t0

    # stencil roofline: the batched fine launch of one iteration (63 fields)
    B = N - 1
    log(f"stencil timing: {B} x {n}^3, {n_f} steps")
    if U_ref is not None:
        xin = U_ref[:B].clone()
    elif not args.stencil_only:
        xin = torch.stack([u0 * (1.0 + 0.01 * i) for i in range(B)])
    else:
        xin = torch.stack([u0 * (1.0 + 0.01 * i) for i in range(B)])
    xout = torch.empty_like(xin)
    items = [dict(prob=prob, dt=dt, n_steps=n_f, u_in=xin[i], u_out=xout[i]) for i in range(B)]
    pr.pr_fine_propagate(ctx, items)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 2
    e0.record(stream)
    for _ in range(reps):
        pr.pr_fine_propagate(ctx, items)
    e1.record(stream)
    torch.cuda.synchronize()
    fine_ms = e0.elapsed_time(e1) / reps
    launches = n_f
    avg_launch_s = fine_ms * 1e-3 / launches
    # algorithmic bytes of one fused RK4 step: read y and write y_new once
    # per point (8 + 8 B in FP64, 4 + 4 B in FP32); halo re-reads and LDS
    # traffic are not counted
    bytes_per_launch = (8 if f32 else 16) * ng * B
    achieved = bytes_per_launch / avg_launch_s / 1e9
    stencil_gpts = B * ng * n_f / (fine_ms * 1e-3) / 1e9
    kname = pr.fine_kernel_name(ctx, prec, n, B) or "k_rk4_fused<double>"
    copy_gbs, runtime_copy_gbs = copy_bandwidth(stream)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(kname, src=stencil_src_of(kname),
                                            profile=stencil_profile_of(kname)),
                "kernel": kname, "avg_launch_us": round(avg_launch_s * 1e6, 2),
                "bytes_per_launch": bytes_per_launch,
                "copy_kernel_gbs": copy_gbs,
                "runtime_copy_gbs": runtime_copy_gbs,
                "frac_of_copy": round(achieved / max(copy_gbs, runtime_copy_gbs), 4)}
    if args.sweep:
        sweep = {}
        for pol in range(3):
            os.environ["PR_FUSED_CHUNK"] = str(pol)
            for cfg in range(FUSED_TILINGS):
                os.environ["PR_FUSED_CFG"] = str(cfg)
                pr.pr_fine_propagate(ctx, items)
                e0.record(stream)
                pr.pr_fine_propagate(ctx, items)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                t = pr.pr_fine_tuned(ctx, prec, n, B, blocked=True)
                key = "%dx%dx%d%s/chunks%d" % (t[:3] + ("b22" if t[3] else "", pol))
                sweep[key] = round(B * ng * n_f / (ms * 1e-3) / 1e9, 2)
                log(f"  tiling {key}: {sweep[key]} GPts/s")
        del os.environ["PR_FUSED_CFG"]
        del os.environ["PR_FUSED_CHUNK"]
        roofline["sweep_gpts"] = sweep
    del xin, xout
    if args.stencil_only:
        # calibration copy of known size for the PMC byte counters: 1 GiB read
        # and 1 GiB written by one copy kernel
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"stencil_gpts": stencil_gpts, "roofline": roofline,
                          "calibration_copy_bytes": a.numel() * 8}))
        ctx.close()
        return

    def one_solve():
        U, rep = pr.pr_parareal_solve(ctx, prob, opts, u0, U_ref=U_ref)
        return U, rep

    for i in range(args.warmup):
        log(f"warmup solve {i}")
        one_solve()
    torch.cuda.synchronize()
    reps_out = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        log(f"timed solve {i}")
        _, rep = one_solve()
        reps_out.append(rep)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    updates = sum(r.fine_updates for r in reps_out)
    value = updates / el / 1e9
    rep = reps_out[-1]
    t_to = None
    for k, e in enumerate(rep.err):
        if e <= 1e-6:
            t_to = rep.t_iter[k]
            break

    out = {
        "metric": "fine-stencil GPts/s + %HBM roofline; parareal time to 1e-6 rel L2; p99 latency",
        "value": round(value, 3),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "flow": "kolmogorov k_f=4", "kappa": w.problem.kappa,
                   "T": opts.T, "N": N, "dt": opts.dt, "n_f": n_f, "cap": opts.cap,
                   "tol": opts.tol, "parallelism": "time subintervals batched on 1 GPU"},
        "iters": rep.iters,
        "converged": rep.converged,
        "err_final": rep.err[-1] if rep.err else None,
        "parareal_time_to_1e-6_s": t_to,
        "serial_fine_s": round(serial_s, 4) if serial_s is not None else None,
        "stencil_gpts": round(stencil_gpts, 2),
        "t_phase_s": {k: round(v, 4) for k, v in rep.t_phase.items()},
        "err_history": [float("%.3e" % e) for e in rep.err],
        "jump_history": [float("%.3e" % e) for e in rep.jump],
        "m0": rep.m0,
        "roofline": roofline,
    }
    # The timed solves prepare the next part of each sweep wave on a second
    # stream, so their phase times overlap and each includes the other's
    # contention. The paper's per-term estimate takes them from one more
    # (untimed) solve with that overlap off.
    if serial_s is not None:
        log("solve without the second stream, for the per-phase estimate")
        old = os.environ.get("PR_SWEEP_PARTS")
        os.environ["PR_SWEEP_PARTS"] = "1"
        try:
            _, rep1 = one_solve()
        finally:
            if old is None:
                del os.environ["PR_SWEEP_PARTS"]
            else:
                os.environ["PR_SWEEP_PARTS"] = old
        out["t_phase_s_serial_streams"] = {k: round(v, 4) for k, v in rep1.t_phase.items()}
        out["paper_projection"] = paper_projection(rep1, serial_s, N)
    else:
        out["paper_projection"] = None
    if args.serve_requests > 0:
        del U_ref
        torch.cuda.empty_cache()
        out["serving"] = serving_sample(pr, ctx, budget, args.serve_requests)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        log("oracle phase times, 32^3 workload")
        out["cpu_baseline"]["oracle_abc32_solve"] = oracle_c1_phases()
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
