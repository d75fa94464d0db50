"""Seeded synthetic workloads shared by the tests, the bench and the oracle runs.

This module holds only the *inputs*: lattice sizes, connectivity, decay
exponents, seeds, temperature ladders and run lengths.  It contains none of
the method's arithmetic (no graph sampling, no colouring, no dynamics), so
both the oracle and the GPU library can be fed from it without sharing code.

The paper's workloads are themselves synthetic random graphs (Sec. 2,
Eq. Levyi; Sec. 4 run parameters); no dataset is involved.  Every graph is
defined by (L, z, rho, seed) and every initial state by (seed, slot, site)
through the counter-based generator each side implements on its own.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np


def linear_ladder(t_min: float, t_max: float, n: int) -> np.ndarray:
    """n temperatures linearly spaced in [t_min, t_max], both ends included."""
    if n == 1:
        return np.array([t_min], dtype=np.float64)
    return np.array([t_min + k * (t_max - t_min) / (n - 1) for k in range(n)], dtype=np.float64)


@dataclass
class Sample:
    L: int
    rho: float
    seed: int
    z: int = 6


@dataclass
class Workload:
    name: str
    samples: List[Sample]
    T: np.ndarray               # temperature ladder, shared by all samples
    n_sweeps: int
    n_or: int = 5               # OR sub-sweeps per sweep (1 Metropolis + n_or OR)
    pt_every: int = 1           # 0 = no parallel tempering
    meas_every: int = 32
    precision: str = "fix16"    # "fp64" or "fix16"
    note: str = ""

    @property
    def n_T(self) -> int:
        return int(self.T.shape[0])

    @property
    def spins(self) -> int:
        return sum(s.L * s.L for s in self.samples)

    def updates_per_sweep(self) -> int:
        return self.spins * self.n_T * (1 + self.n_or)


def plain_fp64_l16() -> Workload:
    """One L=16 graph, z=6, rho=3.5, seed 1, T in {0.8,1.2,1.6,2.0}, no PT,
    1e4 sweeps of 1 Metropolis + 5 OR, measurement every sweep."""
    return Workload("levy_L16_rho3.5_T4_fp64", [Sample(16, 3.5, 1)],
                    np.array([0.8, 1.2, 1.6, 2.0]), n_sweeps=10_000, pt_every=0,
                    meas_every=1, precision="fp64")


def batch_l128() -> Workload:
    """64 samples of L=128, rho=3.5, 16 T in [1.0,2.5], PT every sweep."""
    return Workload("levy_64xL128_rho3.5_T16", [Sample(128, 3.5, s) for s in range(64)],
                    linear_ladder(1.0, 2.5, 16), n_sweeps=20_000, pt_every=1)


def uneven_sizes() -> Workload:
    """128 samples: L = {32,64,128,256}[s // 32], rho = {2.5,3.5,4.5}[s % 3],
    32 T in [0.8,3.0], PT every sweep, one launch."""
    Ls, rhos = (32, 64, 128, 256), (2.5, 3.5, 4.5)
    return Workload("levy_128x_unevenL_T32", [Sample(Ls[s // 32], rhos[s % 3], s) for s in range(128)],
                    linear_ladder(0.8, 3.0, 32), n_sweeps=10_000, pt_every=1)


def headline_l256() -> Workload:
    """64 samples of L=256, rho=3.5, 24 T in [1.0,2.5], PT every sweep, 16-bit angles."""
    return Workload("levy_64xL256_rho3.5_T24", [Sample(256, 3.5, s) for s in range(64)],
                    linear_ladder(1.0, 2.5, 24), n_sweeps=50_000, pt_every=1)


def large_l512() -> Workload:
    """32 samples of L=512, rho=2.5, 16 T in [1.5,3.5], PT every sweep, 16-bit angles."""
    return Workload("levy_32xL512_rho2.5_T16", [Sample(512, 2.5, s) for s in range(32)],
                    linear_ladder(1.5, 3.5, 16), n_sweeps=20_000, pt_every=1)


ALL = {
    "plain_fp64_l16": plain_fp64_l16,
    "batch_l128": batch_l128,
    "uneven_sizes": uneven_sizes,
    "headline_l256": headline_l256,
    "large_l512": large_l512,
}
