"""Continuous-batching request loop over incremental parareal solves.

Requests (a problem, its parareal options and an initial field) arrive at
given times. The loop

* admits queued requests in arrival order while the device budget holds
  them: a request is admitted when its full-width footprint (pr_footprint)
  fits beside the live solves, or when nothing is live (it then runs with
  narrower waves); pr_solve_begin's PR_ENOMEM keeps it queued;
* advances every live solve by one parareal iteration per step
  (pr_solve_step_batch: the fine solves and per-subinterval POD of all live
  solves share launches);
* retires solves as they stop (pr_solve_end) and records arrival-to-result
  latency.

Every solve's snapshots, bases and states stay on the device from admission
to retirement. The loop is host code only; all arithmetic runs in libpr.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, List, Optional

from . import (PrError, pr_footprint, pr_solve_begin, pr_solve_end, pr_solve_state,
               pr_solve_step_batch)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds after the loop starts
    prob: object              # pr_grid_problem
    opts: object              # parareal options (workloads.PararealOpts-like)
    make_u0: Callable         # () -> device FP64 tensor of N_g values
    result: object = None     # device FP64 state at T once completed


@dataclasses.dataclass
class Completed:
    rid: int
    arrival: float
    admitted: float
    finished: float
    iters: int
    status: int
    n: int
    N: int
    fine_updates: float = 0.0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class ServeStats:
    completed: List[Completed]
    wall: float
    steps: int
    max_live: int
    mean_live: float

    def latencies(self, skip: int = 0) -> List[float]:
        done = sorted(self.completed, key=lambda c: c.rid)[skip:]
        return [c.latency for c in done]

    @staticmethod
    def percentile(xs: List[float], q: float) -> Optional[float]:
        """Nearest-rank percentile."""
        if not xs:
            return None
        s = sorted(xs)
        k = max(0, min(len(s) - 1, int(-(-q * len(s) // 100)) - 1))
        return s[k]


def serve(ctx, requests: List[Request], budget_bytes: int, max_live: int = 16,
          log: Optional[Callable[[str], None]] = None) -> ServeStats:
    """Run the request loop until every request has completed."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    queue: collections.deque = collections.deque()
    live = []          # (handle, request, admitted time, footprint)
    completed: List[Completed] = []
    t0 = time.perf_counter()
    steps = 0
    live_sum = 0
    peak = 0
    while pending or queue or live:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.popleft())
        # admission, in arrival order
        while queue and len(live) < max_live:
            r = queue[0]
            need = pr_footprint(r.prob, r.opts)
            held = sum(f for _, _, _, f in live)
            if live and held + need > budget_bytes:
                break
            try:
                h = pr_solve_begin(ctx, r.prob, r.opts, r.make_u0())
            except PrError as e:
                if e.name == "PR_ENOMEM" and live:
                    break
                raise
            queue.popleft()
            live.append((h, r, time.perf_counter() - t0, need))
            if log:
                log(f"admit {r.rid} n={r.prob.n} N={r.opts.N} live={len(live)}")
        if not live:
            if pending:
                time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
            continue
        peak = max(peak, len(live))
        pr_solve_step_batch(ctx, [h for h, _, _, _ in live])
        steps += 1
        live_sum += len(live)
        keep = []
        for h, r, t_adm, need in live:
            if h.done:
                # the result handed back: the state at T
                r.result = pr_solve_state(ctx, h, int(r.opts.N))
                _, rep = pr_solve_end(ctx, h, U_out=False)
                t = time.perf_counter() - t0
                completed.append(Completed(r.rid, r.arrival, t_adm, t, rep.iters, rep.status,
                                           r.prob.n, int(r.opts.N), rep.fine_updates))
                if log:
                    log(f"done {r.rid} iters={rep.iters} status={rep.status} "
                        f"latency={t - r.arrival:.2f}s")
            else:
                keep.append((h, r, t_adm, need))
        live = keep
    wall = time.perf_counter() - t0
    return ServeStats(completed, wall, steps, max_live=peak, mean_live=live_sum / max(steps, 1))
