"""ctypes view of libpr.so (include/pr.h). Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_double, c_int, c_size_t, c_void_p, c_char_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpr.so")

PR_OK = 0
STATUS = {0: "PR_OK", -1: "PR_EINVAL", -2: "PR_ENOMEM", -3: "PR_EDEVICE", -4: "PR_EUNSTABLE",
          -5: "PR_ENOTCONV", -6: "PR_ENUMERIC", -7: "PR_EBUSY"}

PR_FLOW_UNIFORM, PR_FLOW_ABC, PR_FLOW_KOLMOGOROV = 0, 1, 2
PR_FLOW_KOLMOGOROV_T, PR_FLOW_ABC_T = 3, 4
PR_F64, PR_MIXED = 0, 1
PR_MODE_ADAPTIVE, PR_MODE_FIXED_POD, PR_MODE_COARSE_GRID = 0, 1, 2


class pr_grid_problem(Structure):
    _fields_ = [("n", c_int), ("L", c_double), ("kappa", c_double), ("flow", c_int),
                ("fp", c_double * 3), ("precision", c_int)]


class pr_fine_item(Structure):
    _fields_ = [("prob", POINTER(pr_grid_problem)), ("dt", c_double), ("n_steps", c_int),
                ("u_in", c_void_p), ("u_out", c_void_p), ("snap_every", c_int),
                ("snaps", c_void_p), ("t0", c_double)]


class pr_pod_item(Structure):
    _fields_ = [("prob", POINTER(pr_grid_problem)), ("n_blocks", c_int),
                ("blocks", POINTER(c_void_p)), ("block_cols", POINTER(c_int)),
                ("block_valid", POINTER(c_void_p)), ("gamma", c_double), ("cap", c_int),
                ("force_m", c_int), ("R_out", c_void_p), ("m_out", c_void_p),
                ("lambda_out", c_void_p)]


class pr_coarse_item(Structure):
    _fields_ = [("prob", POINTER(pr_grid_problem)), ("R", c_void_p), ("cap", c_int),
                ("m", c_void_p), ("u_aug", c_void_p), ("n_in", c_int), ("u_in", c_void_p * 2),
                ("dT_total", c_double), ("n_c", c_int), ("dt_hint", c_double),
                ("u_out", c_void_p * 2), ("beta_out", c_void_p), ("n_c_out", c_void_p),
                ("t0", c_double)]


class pr_parareal_opts(Structure):
    _fields_ = [("T", c_double), ("N", c_int), ("dt", c_double), ("dM", c_int),
                ("gamma1", c_double), ("gamma2", c_double), ("gamma3", c_double),
                ("cap0", c_int), ("cap", c_int), ("ml", c_int), ("p", c_int),
                ("coarse_ratio", c_int), ("tol", c_double), ("max_iter", c_int),
                ("mode", c_int), ("diag", c_int), ("n_warm", c_int), ("U_ref", c_void_p)]


class pr_report(Structure):
    _fields_ = [("iters", c_int), ("converged", c_int), ("n_f", c_int), ("dM", c_int),
                ("n_s", c_int), ("n_c", c_int), ("n_sub", c_int), ("m0", c_int),
                ("jump", POINTER(c_double)), ("err", POINTER(c_double)),
                ("t_iter", POINTER(c_double)), ("ranks", POINTER(c_int)),
                ("t_phase", c_double * 5), ("fine_updates", c_double), ("seconds", c_double),
                ("gap_fine", POINTER(c_double)), ("gap_ref", POINTER(c_double)),
                ("basis_orth", POINTER(c_double))]


class pr_plan_info(Structure):
    _fields_ = [("n_sub", c_int), ("n_f", c_int), ("dt", c_double), ("dM", c_int),
                ("n_s", c_int), ("n_c", c_int), ("max_iter", c_int)]


EXPORTS = ["pr_ctx_create", "pr_ctx_destroy", "pr_last_error", "pr_ctx_scratch_bytes",
           "pr_fine_propagate", "pr_fine_tuned", "pr_gram", "pr_gram_noalloc", "pr_pod_build", "pr_coarse_propagate",
           "pr_parareal_solve", "pr_plan", "pr_footprint", "pr_solve_begin", "pr_solve_step_batch",
           "pr_solve_state", "pr_solve_done", "pr_solve_bytes", "pr_solve_end"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libpr.so (built in-tree by paper_2601_10981_amd.build). There is
    no fallback: a missing library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpr.so not found at {path}; run paper_2601_10981_amd.build.build()")
    # torch bundles its own HIP runtime (soname libamdhip64.so.7). Importing
    # it first makes libpr's libamdhip64.so.7 dependency bind to that same
    # runtime instead of loading a second one from /opt/rocm, which would leave
    # one of the two without devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    lib.pr_ctx_create.argtypes = [c_int, c_size_t, POINTER(c_void_p)]
    lib.pr_ctx_create.restype = c_int
    lib.pr_ctx_destroy.argtypes = [c_void_p]
    lib.pr_ctx_destroy.restype = None
    lib.pr_last_error.argtypes = [c_void_p]
    lib.pr_last_error.restype = c_char_p
    lib.pr_ctx_scratch_bytes.argtypes = [c_void_p]
    lib.pr_ctx_scratch_bytes.restype = c_size_t
    lib.pr_fine_propagate.argtypes = [c_void_p, c_int, POINTER(pr_fine_item), c_void_p]
    lib.pr_fine_propagate.restype = c_int
    lib.pr_fine_tuned.argtypes = [c_void_p, c_int, c_int, c_int, c_int, POINTER(c_int), POINTER(c_int),
                                  POINTER(c_int), POINTER(c_int), POINTER(c_int)]
    lib.pr_fine_tuned.restype = c_int
    lib.pr_gram.argtypes = [c_void_p, POINTER(pr_grid_problem), c_void_p, c_int, c_void_p,
                            c_void_p]
    lib.pr_gram.restype = c_int
    lib.pr_gram_noalloc.argtypes = [c_void_p, POINTER(pr_grid_problem), c_void_p, c_int, c_void_p,
                                    c_void_p]
    lib.pr_gram_noalloc.restype = c_int
    lib.pr_pod_build.argtypes = [c_void_p, c_int, POINTER(pr_pod_item), c_void_p]
    lib.pr_pod_build.restype = c_int
    lib.pr_coarse_propagate.argtypes = [c_void_p, c_int, POINTER(pr_coarse_item), c_void_p]
    lib.pr_coarse_propagate.restype = c_int
    lib.pr_parareal_solve.argtypes = [c_void_p, POINTER(pr_grid_problem),
                                      POINTER(pr_parareal_opts), c_void_p, c_void_p,
                                      POINTER(pr_report), c_void_p]
    lib.pr_parareal_solve.restype = c_int
    lib.pr_plan.argtypes = [POINTER(pr_grid_problem), POINTER(pr_parareal_opts),
                            POINTER(pr_plan_info)]
    lib.pr_plan.restype = c_int
    lib.pr_footprint.argtypes = [POINTER(pr_grid_problem), POINTER(pr_parareal_opts),
                                 POINTER(c_size_t)]
    lib.pr_footprint.restype = c_int
    lib.pr_solve_begin.argtypes = [c_void_p, POINTER(pr_grid_problem), POINTER(pr_parareal_opts),
                                   c_void_p, POINTER(c_void_p), c_void_p]
    lib.pr_solve_begin.restype = c_int
    lib.pr_solve_step_batch.argtypes = [c_void_p, c_int, POINTER(c_void_p), POINTER(c_int),
                                        c_void_p]
    lib.pr_solve_step_batch.restype = c_int
    lib.pr_solve_state.argtypes = [c_void_p, c_void_p, c_int, c_void_p, c_void_p]
    lib.pr_solve_state.restype = c_int
    lib.pr_solve_done.argtypes = [c_void_p]
    lib.pr_solve_done.restype = c_int
    lib.pr_solve_bytes.argtypes = [c_void_p]
    lib.pr_solve_bytes.restype = c_size_t
    lib.pr_solve_end.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(pr_report), c_void_p]
    lib.pr_solve_end.restype = c_int
    _lib = lib
    return lib
