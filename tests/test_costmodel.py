"""The reporting formulas reproduce the paper's own timing tables (Sec. 4):
T_total = T_F + T_U + T_C + N (T_G + T_A) for every adaptive row, T_F + N T_G
for the coarse-grid rows, and the quoted speedups T_F N / (T_total (k + 1))."""
import json
import os

import pytest

from paper_2601_10981_amd import costmodel

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_phase_times.json")))


@pytest.mark.parametrize("row", GOLD["adaptive"], ids=lambda r: f"{r['flow']}-{r['eps']}")
def test_t_total_adaptive_rows(row):
    t = costmodel.t_total(row["T_F"], row["T_U"], row["T_C"], row["T_G"], row["T_A"], GOLD["N"])
    assert abs(t - row["T_total"]) <= 0.011


@pytest.mark.parametrize("row", GOLD["coarse_grid"], ids=lambda r: f"{r['flow']}-{r['eps']}")
def test_t_total_coarse_grid_rows(row):
    t = costmodel.t_total_coarse_grid(row["T_F"], row["T_G"], GOLD["N"])
    assert abs(t - row["T_total"]) <= 0.011


@pytest.mark.parametrize("q", GOLD["speedup_quotes"], ids=lambda r: f"{r['flow']}-{r['eps']}")
def test_quoted_speedups(q):
    row = [r for r in GOLD["adaptive"] if r["flow"] == q["flow"] and r["eps"] == q["eps"]][0]
    s = costmodel.speedup_estimate(row["T_F"], row["T_total"], GOLD["N"], q["iterations_plus_one"] - 1)
    assert abs(s - q["quoted"]) <= 0.2 * 1.0 + 0.02 * q["quoted"]
