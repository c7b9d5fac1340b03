"""Per-iteration cost bookkeeping of the adaptive parareal method (Sec. 3.3
and the experiments of Sec. 4), used to report measured phase times in the
paper's own terms.

  T_total = T_F + T_U + T_C + N (T_G + T_A)          (per iteration, Sec. 4)
  T_total = T_F + N T_G                              (coarse-grid parareal)
  speedup ~= T_F N / (T_total (k + 1))               (Sec. 4 estimate)
  speedup ~= N / ((1 + C_p3 m_max / C_f * dt / DT * N) k_max)   (eq. speedup)

T_F and T_G are per subinterval; T_U, T_C are per iteration; T_A is per
subinterval (sequential).
"""
from __future__ import annotations


def t_total(T_F: float, T_U: float, T_C: float, T_G: float, T_A: float, N: int) -> float:
    return T_F + T_U + T_C + N * (T_G + T_A)


def t_total_coarse_grid(T_F: float, T_G: float, N: int) -> float:
    return T_F + N * T_G


def speedup_estimate(T_F: float, T_total: float, N: int, k: int) -> float:
    """T_F N / (T_total (k + 1)): k + 1 iterations including the cheaper k = 0."""
    return T_F * N / (T_total * (k + 1))


def speedup_model(N: int, k_max: int, m_max: int, Cp3_over_Cf: float, dt: float, DT: float) -> float:
    """Dominant-term model of eq. speedup."""
    return N / ((1.0 + Cp3_over_Cf * m_max * (dt / DT) * N) * k_max)


def phase_report(t_phase: dict, iters: int, n_sub: int) -> dict:
    """Map measured solve totals (seconds summed over the whole solve: F, C,
    U, A, G) onto the paper's per-iteration quantities. On one GPU all
    subintervals' fine solves share the device, so T_F here is the fine time
    per iteration divided by the subintervals propagated."""
    k = max(iters, 1)
    return {
        "T_F_per_iter": t_phase.get("F", 0.0) / k,
        "T_C_per_iter": t_phase.get("C", 0.0) / k,
        "T_U_per_iter": t_phase.get("U", 0.0) / k,
        "T_A_per_iter": t_phase.get("A", 0.0) / k,
        "T_G_per_iter": t_phase.get("G", 0.0) / k,
        "n_sub": n_sub,
    }
