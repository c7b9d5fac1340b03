"""FP64 CPU oracle for the MOR-based adaptive parareal hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product imports this package: only
the tests, the smoke check and the benchmark's CPU-baseline leg may call it.
It shares no code with the HIP path; the only common module is ``workloads``,
which holds seeded input generators and no arithmetic of the method.

The oracle is deliberately plain and slow: numpy FP64, whole-array operations,
no blocking or fusion, each function written from the paper's definitions:

  fd       -- periodic FD operator L and classical RK4 (the fine propagator
              F that replaces the paper's FEM + implicit Euler, Sec. 3.1)
  pod      -- POD_Mode (Algorithm 1, Sec. 3.2 Case I) with the sqrt(lambda)
              rank criterion
  coarse   -- reduced Galerkin system (eq. 8 / eq00), augmentation by the
              interface state (eqaug, eq12, eq13) and the reduced propagator
  parareal -- the adaptive parareal iteration (formula4, Algorithm 2) and the
              serial fine reference used by the error metric (eq. error)

Every function states the passage it follows and the reading taken where the
paper is silent.
"""
from . import fd, pod, coarse, parareal  # noqa: F401
