"""Seeded synthetic inputs for the Allen–Cahn/Cahn–Hilliard solver and its oracle.

This module holds no arithmetic of the method: it only draws initial fields and
describes workloads.  Both the HIP path (through its tests and the benchmark)
and the CPU oracle receive the arrays it returns, so the two sides never share
any code of the method itself.

Array convention: a 2D field has shape (ny, nx) and a 3D field (nz, ny, nx),
C order, x fastest.  Random draws use NumPy's PCG64 ``default_rng(seed)``,
u-noise first, then v-noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Workload", "random_ic", "smooth_ic_2d", "perturbed_pair", "workloads",
    "batched_instances",
]


def random_ic(shape, seed: int, u_mean: float = 0.5, u_amp: float = 0.05,
              v_amp: float = 0.05) -> Tuple[np.ndarray, np.ndarray]:
    """u0 = u_mean + u_amp*U(-1,1), v0 = v_amp*U(-1,1) (Section 4.1 random
    initial data; the 0.5 mean is the benchmark's, the paper uses 0.55)."""
    rng = np.random.default_rng(seed)
    du = rng.uniform(-1.0, 1.0, size=shape)
    dv = rng.uniform(-1.0, 1.0, size=shape)
    return (u_mean + u_amp * du).astype(np.float64), (v_amp * dv).astype(np.float64)


def smooth_ic_2d(nx: int, ny: int, Lx: float = 1.0, Ly: float = 1.0):
    """The smooth periodic initial data of the convergence study (Section 4.1 A):
    u = 0.4(sin^2 2πx + cos^2 2πy) + 0.1, v = 0.4(sin^2 2πx - cos^2 2πy),
    sampled at cell centres."""
    x = (np.arange(nx) + 0.5) * (Lx / nx)
    y = (np.arange(ny) + 0.5) * (Ly / ny)
    X, Y = np.meshgrid(x, y, indexing="xy")
    s = np.sin(2 * np.pi * X) ** 2
    c = np.cos(2 * np.pi * Y) ** 2
    return 0.4 * (s + c) + 0.1, 0.4 * (s - c)


def perturbed_pair(shape, seed: int, amp: float = 0.02, u_mean: float = 0.5,
                   u_amp: float = 0.05, v_amp: float = 0.05):
    """A previous state (u0, v0) and a nearby trial state (u1, v1); both admissible
    (u±v strictly inside (0,1)) for the default amplitudes."""
    u0, v0 = random_ic(shape, seed, u_mean, u_amp, v_amp)
    rng = np.random.default_rng(seed + 7919)
    u1 = u0 + amp * rng.uniform(-1.0, 1.0, size=shape)
    v1 = v0 + amp * rng.uniform(-1.0, 1.0, size=shape)
    return u1, v1, u0, v0


@dataclass
class Workload:
    """One benchmark / parity configuration (all physical and solver settings)."""
    name: str
    dim: int
    n: Tuple[int, int, int]
    bc: str                      # "periodic" or "neumann"
    alpha: float = 1.2
    beta: float = 1.2
    theta: float = 0.1
    gamma: float = 1e-3
    rho: float = 1.0
    S: int = 10
    steps: int = 10
    adaptive: bool = False
    dt_fixed: float = 1e-3
    dt_min: float = 1e-4
    dt_max: float = 1e-1
    eta0: float = 1e4
    sub: Tuple[int, int, int] = (2, 2, 1)
    overlap: int = 1
    precision: str = "fp64"      # "fp64" or "mixed"
    newton_rtol: float = 1e-8
    newton_atol: float = 1e-13
    gmres_rtol: float = 1e-8
    gmres_atol: float = 1e-14
    gmres_restart: int = 30
    seed: int = 0
    u_mean: float = 0.5

    def shape(self):
        nx, ny, nz = self.n
        return (ny, nx) if self.dim == 2 else (nz, ny, nx)

    def initial(self):
        return random_ic(self.shape(), self.seed, u_mean=self.u_mean)

    def to_dict(self):
        return asdict(self)


def workloads():
    """The five benchmark configurations (2D periodic 64^2 parity case, 2D
    periodic 512^2 adaptive FP64 case, 2D Neumann 2048^2 mixed-precision case,
    3D Neumann 128^3 case) plus the batched case through batched_instances()."""
    return {
        "periodic64": Workload("periodic64", 2, (64, 64, 1), "periodic", steps=10,
                               adaptive=False, dt_fixed=1e-3, sub=(2, 2, 1), overlap=1),
        "periodic512": Workload("periodic512", 2, (512, 512, 1), "periodic", steps=200,
                                adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1e4,
                                sub=(8, 8, 1), overlap=2),
        "neumann2048": Workload("neumann2048", 2, (2048, 2048, 1), "neumann", steps=50,
                                adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1e4,
                                sub=(16, 16, 1), overlap=2, precision="mixed"),
        "neumann3d128": Workload("neumann3d128", 3, (128, 128, 128), "neumann", steps=20,
                                 adaptive=True, dt_min=1e-4, dt_max=2.0, eta0=100.0,
                                 sub=(4, 4, 4), overlap=1),
    }


def batched_instances(count: int = 96, base_seed: int = 1000):
    """Independent 2D periodic instances: N uniform over {96,128,192,256},
    theta ~ U(0.08,0.12), gamma ~ U(5e-4,2e-3), seeded noise initial data.
    Instance i draws everything from seed base_seed+i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        n = int(rng.choice([96, 128, 192, 256]))
        theta = float(rng.uniform(0.08, 0.12))
        gamma = float(rng.uniform(5e-4, 2e-3))
        w = Workload(f"inst{i}", 2, (n, n, 1), "periodic", theta=theta, gamma=gamma,
                     steps=10, adaptive=False, dt_fixed=1e-3, seed=base_seed + i)
        out.append(w)
    return out
