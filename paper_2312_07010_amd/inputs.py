"""Seeded synthetic inputs and workload shapes for the Allen-Cahn runs.

This module holds no arithmetic of the scheme.  It only draws initial fields
and instance descriptors from seeded generators, so that the GPU library and
the CPU oracle receive byte-identical inputs.  Node coordinates are passed in
by the caller (each side computes its own layout).  The batched workload's
time steps are defined as half the largest step the stability condition
allows; that formula fixes an input here and takes no part in any step.

Workloads mirror the paper's experiments (Sec. 4): uniform random fields as
in the 1D Dirichlet example, smooth tanh interfaces as in the mean-curvature
examples, and mixed batches of 1D/2D problems.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

HN, HD, P = 0, 1, 2


@dataclass
class Workload:
    name: str
    d: int
    N: List[int]
    L: List[float]
    R: List[float]
    eps: float
    dt: float
    bc: int
    steps: int
    every: int = 100
    ic: str = "uniform"
    lo: float = -0.9
    hi: float = 0.9
    seed: int = 0
    extra: dict = field(default_factory=dict)


# 1D periodic, 256 cells on (-1, 1), eps 0.02, dt 1e-3, 2000 steps.
W1D = Workload("1d_p_256", 1, [256], [-1.0], [1.0], 0.02, 1e-3, P, 2000,
               100, "uniform", -0.05, 0.05, 0)
# 2D Neumann on (0,1)^2 with 1024 x 1024 stored nodes (N = 1022 cells).
W2D = Workload("2d_hn_1024", 2, [1022, 1022], [0.0, 0.0], [1.0, 1.0], 0.01,
               1e-3, HN, 10000, 100, "uniform", -0.9, 0.9, 0)
# 3D periodic 512^3 on (0,1)^3, eps 0.02, dt 5e-4, sphere of radius 0.3.
W3D = Workload("3d_p_512", 3, [512, 512, 512], [0.0] * 3, [1.0] * 3, 0.02,
               5e-4, P, 5000, 100, "sphere", -0.01, 0.01, 0,
               {"radius": 0.3, "center": [0.5, 0.5, 0.5]})
# Adjoint: 2D Neumann 512 x 512 stored nodes (N = 510), eps^2 = 1e-4.
WADJ = Workload("adj_2d_hn_512", 2, [510, 510], [0.0, 0.0], [1.0, 1.0], 0.01,
                1e-3, HN, 1000, 0, "uniform", -0.5, 0.5, 2,
                {"target_seed": 1, "ckpt_every": 32})
WORKLOADS = {w.name: w for w in (W1D, W2D, W3D, WADJ)}


def uniform_field(shape, lo, hi, seed):
    """i.i.d. Uniform[lo, hi] in C order over the stored nodes."""
    return np.random.default_rng(seed).uniform(lo, hi, size=tuple(shape))


def sphere_field(coords, eps, radius, center, noise, seed):
    """tanh((radius - |x - c|)/(sqrt(2) eps)) + Uniform[-noise, noise],
    clipped to [-1, 1] so the maximum-principle hypothesis holds.

    coords: one 1D array of node coordinates per axis (C order)."""
    grids = np.meshgrid(*coords, indexing="ij")
    r2 = sum((g - c) ** 2 for g, c in zip(grids, center))
    base = np.tanh((radius - np.sqrt(r2)) / (np.sqrt(2.0) * eps))
    shape = base.shape
    base = base + np.random.default_rng(seed).uniform(-noise, noise, size=shape)
    return np.clip(base, -1.0, 1.0)


def initial_field(w: Workload, shape, coords=None):
    if w.ic == "uniform":
        return uniform_field(shape, w.lo, w.hi, w.seed)
    if w.ic == "sphere":
        return sphere_field(coords, w.eps, w.extra["radius"], w.extra["center"],
                            w.hi, w.seed)
    raise ValueError(w.ic)


@dataclass
class Instance:
    d: int
    N: int
    eps: float
    bc: int
    dt: float


def batch_instances(count=4096, seed=3, n1=(128, 4096), n2=(32, 512),
                    eps_range=(0.01, 0.05), dt_fraction=0.5):
    """Mixed batch: first half 1D, second half 2D on (0,1)^d; N log-uniform,
    eps uniform, BC uniform over {HN, HD, P}; dt = dt_fraction times the
    largest step allowed by dt <= 1 - 2 d eps^2 dt / dx^2, i.e.
    dt_max = dx^2 / (dx^2 + 2 d eps^2)."""
    root = np.random.SeedSequence(seed)
    kids = root.spawn(count)
    out = []
    for i, ss in enumerate(kids):
        r = np.random.default_rng(ss)
        d = 1 if i < count // 2 else 2
        lo, hi = n1 if d == 1 else n2
        N = int(round(np.exp(r.uniform(np.log(lo), np.log(hi)))))
        eps = float(r.uniform(*eps_range))
        bc = int(r.integers(0, 3))
        dx = 1.0 / N
        dt = dt_fraction * dx * dx / (dx * dx + 2 * d * eps * eps)
        out.append(Instance(d, N, eps, bc, dt))
    return out


def batch_phi0(i, shape, seed=3, lo=-0.9, hi=0.9):
    """Initial field of instance i of a batch: Uniform[lo, hi] from its own
    seed sequence (seed, i)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, i]))
    return rng.uniform(lo, hi, size=tuple(shape))
