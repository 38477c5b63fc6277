"""Seeded synthetic workloads: model parameters and initial fields.

This module holds no arithmetic of the method.  It only names the workloads
(box, grid, contour steps, model constants) and draws their seeded initial
fields with numpy, so that the GPU path, the CPU oracle, the tests and the
benchmark all start from identical inputs.

The paper evaluates on synthetic, randomly seeded fields, not on a dataset
(Sec. V: lamellar and gyroid diblock melts whose fields start from
decorrelated random noise).  Every field here is drawn from
``numpy.random.default_rng(seed)`` in the fixed order Re w+, Im w+, Re w-,
Im w-, C-order [nx][ny][nz].
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n: Tuple[int, int, int]
    L: Tuple[float, float, float]
    ns: int
    f: float
    chiN: float
    C: float = 1.0
    seed: int = 1204
    # field distribution: (sigma Re w+, sigma Im w+, sigma Re w-, sigma Im w-)
    sigma: Tuple[float, float, float, float] = (0.1, 0.02, 0.1, 0.02)
    cosine_wm: float = 0.0          # amplitude of a cos(2 pi x / Lx) added to w-
    dt: float = 0.01
    noise: bool = True
    steps: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def scaled(self, n: Tuple[int, int, int], ns: Optional[int] = None) -> "Workload":
        """Same model and field distribution on another grid (box edges scale with n)."""
        L = tuple(self.L[a] * n[a] / self.n[a] for a in range(3))
        return replace(self, n=tuple(n), L=L, ns=self.ns if ns is None else ns)


def fields(w: Workload, seed: Optional[int] = None):
    """Seeded initial (w_plus, w_minus) as complex128 arrays of shape n."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    shape = tuple(w.n)
    s = w.sigma
    draws = [rng.standard_normal(shape) * sd if sd > 0 else np.zeros(shape) for sd in s]
    wp = draws[0] + 1j * draws[1]
    wm = draws[2] + 1j * draws[3]
    if w.cosine_wm:
        x = np.arange(shape[0]).reshape(-1, 1, 1) / shape[0]
        wm = wm + w.cosine_wm * np.cos(2.0 * np.pi * x)
    return np.ascontiguousarray(wp), np.ascontiguousarray(wm)


# Lamellar benchmark of Sec. V (f_A = 0.5, chi N = 14.0, cubic cell 10.89 R_g),
# at the paper's largest grid, 128^3, with 100 contour steps (the paper's own
# memory example in Sec. IV.C).  Random complex fields.
LAM128 = Workload("lam128", (128, 128, 128), (10.89,) * 3, 100, 0.5, 14.0, C=1.0, seed=1204)
# Gyroid parameters of Sec. V (f_A = 0.4, chi N = 14.4, cell 8.82 R_g).
GYR128 = Workload("gyr128", (128, 128, 128), (8.82,) * 3, 100, 0.4, 14.4, C=1.0, seed=1204)

# Deterministic relaxation: 16^3, L = 4, 50 steps, w+ = 0, real w- ~ N(0, 0.1).
SCFT16 = Workload("scft16", (16, 16, 16), (4.0,) * 3, 50, 0.5, 15.0, C=1.0, seed=1205,
                  sigma=(0.0, 0.0, 0.1, 0.0), dt=0.05, noise=False, steps=100)
# Complex Langevin: 64^3, L = 6, 100 steps, C = 50, complex fields.
CL64 = Workload("cl64", (64, 64, 64), (6.0,) * 3, 100, 0.4, 20.0, C=50.0, seed=1206,
                sigma=(0.2, 0.05, 0.2, 0.05), dt=0.01, noise=True, steps=1000)
# Gradient state: 96^3, L = 5.5, 128 steps, f = 0.3 (junction node inside a step).
GRAD96 = Workload("grad96", (96, 96, 96), (5.5,) * 3, 128, 0.3, 18.0, C=1.0, seed=1207,
                  sigma=(0.0, 0.0, 0.05, 0.0), cosine_wm=1.0, noise=False)
# Large single-GPU run: 256^3, L = 16, 200 steps, C = 100.
CL256 = Workload("cl256", (256, 256, 256), (16.0,) * 3, 200, 0.35, 22.0, C=100.0, seed=1209,
                 sigma=(0.2, 0.05, 0.2, 0.05), dt=0.005, noise=True, steps=200)

# Edwards homopolymer solution (Eq. (2)) on the benchmark grid: 128^3, the
# lamellar cell, 100 contour steps, C = 1, excluded volume B = 1; the one field
# omega is the w+ draw (w- is not used).
EDW128 = Workload("edw128", (128, 128, 128), (10.89,) * 3, 100, 0.5, 1.0, C=1.0, seed=1210,
                  sigma=(0.1, 0.02, 0.0, 0.0), extra={"model": "edwards", "B": 1.0})

WORKLOADS = {w.name: w for w in (LAM128, GYR128, SCFT16, CL64, GRAD96, CL256, EDW128)}


def batch_replicas(count: int = 256, seed: int = 1208):
    """Uneven replica set: grids from {24,32,40,48}^3 with L = 0.125 N, Ns in
    [40, 80], chi N in [12, 25], f in [0.3, 0.5], C = 50, dt = 0.01."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        n = int(rng.choice([24, 32, 40, 48]))
        ns = int(rng.integers(40, 81))
        chiN = float(rng.uniform(12.0, 25.0))
        f = float(rng.uniform(0.3, 0.5))
        out.append(Workload(f"rep{r}", (n, n, n), (0.125 * n,) * 3, ns, f, chiN, C=50.0,
                            seed=seed * 1000 + r, sigma=(0.1, 0.02, 0.1, 0.02), dt=0.01,
                            noise=True, steps=500))
    return out
