"""Per-iteration cost bookkeeping of the adaptive parareal method (Sec. 3.3
and the experiments of Sec. 4), used to report measured phase times in the
paper's own terms.

  T_total = T_F + T_U + T_C + N (T_G + T_A)          (per iteration, Sec. 4)
  T_total = T_F + N T_G                              (coarse-grid parareal)
  speedup ~= T_F N / (T_total (k + 1))               (Sec. 4 estimate)

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
