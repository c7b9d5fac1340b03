"""Seeded synthetic workloads for the adaptive parareal hot path.

This module holds only problem sizes and seeded random inputs. It contains
none of the method's arithmetic (no stencil, no POD, no propagator), so both
the FP64 CPU oracle and the HIP path can draw identical inputs from it without
sharing any computation.

The paper (Sec. 4) solves forced advection-diffusion with FEM on 2,097,152
DOF; its workloads are analytic PDE set-ups, not datasets. The configurations
below are the finite-difference stand-ins: periodic [0, 2*pi)^3 grids with
steady ABC or Kolmogorov shear velocity and a seeded initial field.

All fields are generated once on the host in FP64 with numpy's PCG64, laid
out [x][y][z] with z fastest (C order of an (n, n, n) array).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

TWO_PI = 2.0 * math.pi

FLOW_UNIFORM = 0
FLOW_ABC = 1
FLOW_KOLMOGOROV = 2
FLOW_KOLMOGOROV_T = 3   # the Kolmogorov flow of Sec. 4: B(t) and forcing f(t)
FLOW_ABC_T = 4          # the ABC flow of Sec. 4 with phase sin(w t), forced

PREC_F64 = 0
PREC_MIXED = 1

MODE_ADAPTIVE = 0    # Algorithm 2: local-in-time POD bases rebuilt every iteration
MODE_FIXED_POD = 1   # "Parareal-I" of Sec. 4: the k = 0 POD basis for every iteration
MODE_COARSE_GRID = 2  # "Parareal-II" of Sec. 4: the equation on the n/2 grid as coarse propagator


@dataclasses.dataclass(frozen=True)
class Problem:
    """A periodic advection-diffusion problem on an n^3 node-centred grid.

    flow parameters ``fp``:
      ABC:        (A, B, C)
      KOLMOGOROV: (amplitude, k_f, unused)
      UNIFORM:    (c_x, c_y, c_z)
      KOLMOGOROV_T, ABC_T: (a_v, a_f, w) -- velocity and forcing scales and
                  the frequency of the time dependence (Sec. 4: 1, 1, 1)
    """
    n: int
    kappa: float
    flow: int
    fp: tuple
    precision: int = PREC_F64
    L: float = TWO_PI


@dataclasses.dataclass(frozen=True)
class PararealOpts:
    """Parameters of the adaptive parareal solve (the parameter list that
    opens Algorithm 2, plus rank caps and a stopping tolerance)."""
    T: float
    N: int
    dt: float
    dM: int = 0              # 0: ceil(n_f / 16)
    gamma1: float = 1.0 - 5.0e-6
    gamma2: float = 1.0 - 5.0e-6
    gamma3: float = 1.0 - 2.0e-8
    cap0: int = 10
    cap: int = 10
    ml: int = 1
    p: int = 1
    coarse_ratio: int = 10
    tol: float = 1e-8
    max_iter: int = 0        # 0: N - 1
    mode: int = MODE_ADAPTIVE
    diag: int = 0            # 1: record the coarse-gap diagnostics (Sec. 4, dT = delta t runs)
    n_warm: int = 1          # subintervals in the warm-up window [0, T_0]: T_0 = n_warm DeltaT


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    problem: Problem
    opts: PararealOpts
    seed: int
    init: str                # "blob" or "fourier"


def _canonical_wavevectors(kmax: float) -> np.ndarray:
    """All integer k != 0 with |k| <= kmax, one representative per +-k pair
    (first non-zero component positive), in lexicographic order."""
    r = int(math.floor(kmax))
    out = []
    for a in range(-r, r + 1):
        for b in range(-r, r + 1):
            for c in range(-r, r + 1):
                if a == 0 and b == 0 and c == 0:
                    continue
                if a * a + b * b + c * c > kmax * kmax:
                    continue
                first = a if a != 0 else (b if b != 0 else c)
                if first < 0:
                    continue
                out.append((a, b, c))
    return np.array(out, dtype=np.int64)


def fourier_modes(seed: int, n_modes: int = 16, kmax: float = 8.0):
    """The seeded draw of fourier_field: wavevectors (n_modes x 3 ints) and
    phases theta ~ U[0, 2pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = _canonical_wavevectors(kmax)
    pick = rng.choice(len(ks), size=n_modes, replace=False)
    theta = rng.uniform(0.0, TWO_PI, size=n_modes)
    return ks[pick], theta


def fourier_field(n: int, seed: int, n_modes: int = 16, kmax: float = 8.0,
                  L: float = TWO_PI) -> np.ndarray:
    """Sum of ``n_modes`` distinct random Fourier modes with |k| <= kmax and
    amplitude |k|^-2: phi = sum_k |k|^-2 cos(k.x + theta_k), theta ~ U[0, 2pi)."""
    ks, theta = fourier_modes(seed, n_modes, kmax)
    x = np.arange(n, dtype=np.float64) * (L / n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    scale = TWO_PI / L
    phi = np.zeros((n, n, n), dtype=np.float64)
    for k, th in zip(ks, theta):
        k = k.astype(np.float64)
        amp = 1.0 / float(k @ k)
        phi += amp * np.cos(scale * (k[0] * X + k[1] * Y + k[2] * Z) + th)
    return phi


def fourier_field_device(n: int, seed: int, device, n_modes: int = 16, kmax: float = 8.0,
                         L: float = TWO_PI):
    """fourier_field evaluated with torch on ``device`` (the same seeded
    draw; values agree with the host version to FP64 rounding). For large
    grids in serving runs, where host generation would dominate."""
    import torch
    ks, theta = fourier_modes(seed, n_modes, kmax)
    x = torch.arange(n, dtype=torch.float64, device=device) * (L / n)
    scale = TWO_PI / L
    phi = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    for k, th in zip(ks, theta):
        amp = 1.0 / float(k @ k)
        arg = (scale * float(k[0]) * x).view(n, 1, 1) + (scale * float(k[1]) * x).view(1, n, 1) \
            + (scale * float(k[2]) * x).view(1, 1, n)
        phi += amp * torch.cos(arg + float(th))
    return phi


def blob_field(n: int, seed: int, sigma: float = 0.5, noise: float = 1e-3,
               L: float = TWO_PI) -> np.ndarray:
    """Gaussian blob of width sigma at a seeded centre in [0, L)^3 (minimum
    image periodic distance) plus ``noise`` * U(-1, 1) seeded noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centre = rng.uniform(0.0, L, size=3)
    x = np.arange(n, dtype=np.float64) * (L / n)
    d2 = np.zeros((n, n, n), dtype=np.float64)
    for axis in range(3):
        d = x - centre[axis]
        d = d - L * np.round(d / L)
        shape = [1, 1, 1]
        shape[axis] = n
        d2 = d2 + (d * d).reshape(shape)
    phi = np.exp(-d2 / (2.0 * sigma * sigma))
    phi += noise * rng.uniform(-1.0, 1.0, size=(n, n, n))
    return phi


def random_field(n: int, seed: int) -> np.ndarray:
    """Plain U(-1, 1) field (used for operator-level tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=(n, n, n))


def random_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=(rows, cols))


def initial_field(w: Workload, n: Optional[int] = None) -> np.ndarray:
    n = w.problem.n if n is None else n
    if w.init == "blob":
        return blob_field(n, w.seed, L=w.problem.L)
    return fourier_field(n, w.seed, L=w.problem.L)


# The five configurations of the benchmark family. Names state what they are.
ABC_32_F64 = Workload(
    name="abc32_f64_T1_N8",
    problem=Problem(n=32, kappa=0.05, flow=FLOW_ABC, fp=(1.0, 1.0, 1.0)),
    opts=PararealOpts(T=1.0, N=8, dt=2e-3, cap0=10, cap=10, tol=1e-8),
    seed=1, init="blob")

KOL_128_F64 = Workload(
    name="kolmogorov128_f64_T10_N64",
    problem=Problem(n=128, kappa=0.01, flow=FLOW_KOLMOGOROV, fp=(1.0, 4.0, 0.0)),
    opts=PararealOpts(T=10.0, N=64, dt=1e-3, cap0=20, cap=20, tol=1e-8),
    seed=2, init="fourier")

ABC_256_MIXED = Workload(
    name="abc256_mixed_T50_N128",
    problem=Problem(n=256, kappa=0.005, flow=FLOW_ABC, fp=(1.0, 1.0, 1.0),
                    precision=PREC_MIXED),
    opts=PararealOpts(T=50.0, N=128, dt=5e-4, cap0=10, cap=20, tol=1e-6),
    seed=3, init="fourier")

STANDARD = [ABC_32_F64, KOL_128_F64, ABC_256_MIXED]
BY_NAME = {w.name: w for w in STANDARD}


def ensemble(count: int = 48, seed_base: int = 4000,
             grids=(64, 96, 128, 192)) -> List[Workload]:
    """Batched ensemble of independent instances: grid from ``grids``, ABC or
    Kolmogorov (k_f in 1..4) with probability 1/2, kappa log-uniform in
    [0.005, 0.1], T ~ U[1, 20], N ~ U{16..64}, mixed precision, Fourier
    initial field. Instance i uses seed seed_base + i."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed_base + i))
        n = int(rng.choice(np.array(grids)))
        if rng.uniform() < 0.5:
            flow, fp = FLOW_ABC, (1.0, 1.0, 1.0)
        else:
            flow, fp = FLOW_KOLMOGOROV, (1.0, float(rng.integers(1, 5)), 0.0)
        kappa = float(math.exp(rng.uniform(math.log(0.005), math.log(0.1))))
        T = float(rng.uniform(1.0, 20.0))
        N = int(rng.integers(16, 65))
        out.append(Workload(
            name=f"ensemble{i}",
            problem=Problem(n=n, kappa=kappa, flow=flow, fp=fp,
                            precision=PREC_MIXED),
            opts=PararealOpts(T=T, N=N, dt=0.0, cap0=10, cap=20, tol=1e-6),
            seed=seed_base + i, init="fourier"))
    return out


def serving_requests(count: int = 256, seed_base: int = 5000,
                     grids=tuple(range(64, 257, 32))) -> List[Workload]:
    """Requests of the serving stream: as ``ensemble`` (flow, kappa, T, N,
    automatic dt, mixed precision) with the grid uniform over 64..256 in
    steps of 32 and tolerance 1e-6. Request i uses seed seed_base + i."""
    out = ensemble(count, seed_base, grids)
    return [dataclasses.replace(w, name=f"request{i}") for i, w in enumerate(out)]


def poisson_arrivals(count: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream of ``rate``
    requests per second: cumulative sums of exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
