"""The C ABI library loads and exports every entry point include/pr.h
declares (no device calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2601_10981_amd", "libpr.so")


def _declared():
    src = open(os.path.join(ROOT, "include", "pr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2601_10981_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ["pr_fine_propagate", "pr_pod_build", "pr_coarse_propagate", "pr_parareal_solve",
              "pr_ctx_create", "pr_ctx_destroy", "pr_last_error", "pr_footprint"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_exports():
    from paper_2601_10981_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def test_footprint_is_host_only():
    import workloads as W
    import paper_2601_10981_amd as pr
    w = W.KOL_128_F64
    b = pr.pr_footprint(pr.problem_of(w.problem), w.opts)
    ng = 128 ** 3
    # at least the two state sets, F_n and two slots of stage-1 bases
    assert b >= (2 * 64 + 63) * ng * 8 + 2 * 63 * 20 * ng * 8
    with pytest.raises(pr.PrError) as e:
        pr.pr_footprint(pr.problem_of(w.problem), W.PararealOpts(T=10.0, N=64, dt=10.0))
    assert e.value.name == "PR_EUNSTABLE"


@pytest.mark.parametrize("w", ["abc32", "kol128", "abc256", "ens0", "ens7"])
def test_plan_matches_the_oracle_reading(w):
    """pr_plan (host only) derives n_f, delta_t, dM, n_s and n_c by the same
    readings as the oracle: the step-count rule, the snapshot stride, the
    coarse step rule and, for dt <= 0, the automatic step."""
    import paper_2601_10981_amd as pr
    import workloads as W
    from oracle import coarse, fd, parareal
    wl = {"abc32": W.ABC_32_F64, "kol128": W.KOL_128_F64, "abc256": W.ABC_256_MIXED,
          "ens0": W.ensemble(8)[0], "ens7": W.ensemble(8)[7]}[w]
    plan = pr.pr_plan(pr.problem_of(wl.problem), wl.opts)
    n_f, dt = fd.steps_per_subinterval(wl.opts.T / wl.opts.N,
                                       parareal.requested_dt(wl.problem, wl.opts))
    dM = fd.snapshot_stride(n_f, wl.opts.dM)
    assert plan["n_f"] == n_f and plan["dM"] == dM
    assert plan["dt"] == pytest.approx(dt, rel=1e-15)
    assert plan["n_s"] == n_f // dM + 1
    assert plan["n_c"] == coarse.coarse_steps(n_f, wl.opts.coarse_ratio)
    assert plan["n_sub"] == wl.opts.N - 1



@pytest.mark.parametrize("flow,fp,kappa", [(3, (1.0, 1.0, 1.0), 0.01), (4, (0.7, 1.3, 2.0), 0.05),
                                           (3, (2.5, 0.0, 1.0), 0.0)])
def test_plan_forced_flows_automatic_step(flow, fp, kappa):
    """For the forced flows the automatic step uses sum_d max|v_d| = 6 |a_v|
    (host only, against the oracle's rule)."""
    import paper_2601_10981_amd as pr
    import workloads as W
    from oracle import fd, parareal
    prob = W.Problem(n=64, kappa=kappa, flow=flow, fp=fp)
    opts = W.PararealOpts(T=2.0, N=8, dt=0.0)
    plan = pr.pr_plan(pr.problem_of(prob), opts)
    n_f, dt = fd.steps_per_subinterval(opts.T / opts.N, parareal.requested_dt(prob, opts))
    assert plan["n_f"] == n_f
    assert plan["dt"] == pytest.approx(dt, rel=1e-15)
    assert fd.velocity_bound(flow, fp) == 6.0 * abs(fp[0])

def test_plan_warm_up_window():
    """n_warm subintervals of warm-up leave N - n_warm parareal subintervals
    (host only); a window longer than [0, T] is rejected."""
    import paper_2601_10981_amd as pr
    import workloads as W
    prob = W.Problem(n=32, kappa=0.05, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0))
    for nw in (1, 2, 3):
        opts = W.PararealOpts(T=1.0, N=8, dt=2e-3, n_warm=nw)
        plan = pr.pr_plan(pr.problem_of(prob), opts)
        assert plan["n_sub"] == 8 - nw and plan["max_iter"] == 8 - nw
    # beyond [0, T], and a window whose snapshots (5 x 63 steps every 4) exceed 64
    for nw in (9, 5):
        with pytest.raises(pr.PrError) as e:
            pr.pr_plan(pr.problem_of(prob), W.PararealOpts(T=1.0, N=8, dt=2e-3, n_warm=nw))
        assert e.value.name == "PR_EINVAL"
    # the coarse-grid mode takes no snapshots: any window inside [0, T]
    opts = W.PararealOpts(T=1.0, N=8, dt=2e-3, n_warm=5, mode=W.MODE_COARSE_GRID)
    assert pr.pr_plan(pr.problem_of(prob), opts)["n_sub"] == 3
