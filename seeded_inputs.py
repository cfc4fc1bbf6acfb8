"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module holds workload definitions and random draws only: no part of the
DQMC arithmetic lives here.  Both the oracle (``oracle/``) and the GPU path's
callers draw their inputs from the functions below, so the two sides see
identical Ising fields and Metropolis uniforms.

Recipe
------
* Ising Hubbard-Stratonovich fields: i.i.d. +-1 with probability 1/2 each (a
  hot start), shape ``(L_tau, N)``, site order ``i = (x1*L + x2)*3 + s``,
  drawn from ``numpy.random.default_rng(seed)``.
* Metropolis uniforms: U[0,1) from ``default_rng(seed + 10**6)``, one per
  (sweep, slice, site) in visiting order, shape ``(n_sweeps, L_tau, N)``.
* Batched chains: chain parameters (L, U, beta) drawn from
  ``default_rng(64)``; chain ``c`` uses seed ``4000 + c``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One kagome attractive-Hubbard workload (t=1, periodic boundaries)."""

    name: str
    L: int
    U: float
    beta: float
    dtau: float = 0.1
    t: float = 1.0
    delay_k: int = 32
    n_stab: int = 10
    sweeps: int = 1
    seed: int = 0
    prec: str = "fp64"  # "fp64" | "mixed_f16" | "mixed_bf16"

    @property
    def N(self) -> int:
        return 3 * self.L * self.L

    @property
    def L_tau(self) -> int:
        return int(round(self.beta / self.dtau))


# The five workloads the method is exercised on.
C1 = Workload("kagome-L3-U-4-beta2-fp64-k1", L=3, U=-4.0, beta=2.0, delay_k=1, sweeps=1, seed=3)
C2 = Workload("kagome-L12-U-4-beta8-fp64-k32", L=12, U=-4.0, beta=8.0, delay_k=32, sweeps=10, seed=12)
C3 = Workload("kagome-L18-U-5-beta12-mixed", L=18, U=-5.0, beta=12.0, delay_k=64, sweeps=1, seed=18,
              prec="mixed_f16")
C5 = Workload("kagome-L24-U-4-beta24-mixed", L=24, U=-4.0, beta=24.0, delay_k=128, sweeps=5, seed=24,
              prec="mixed_f16")

WORKLOADS = {w.name: w for w in (C1, C2, C3, C5)}


def batched_chains(n_chains: int = 64, seed: int = 64):
    """Parameters of the batched workload: L in {6,9,12,15}, U in {-3,-4,-5},
    beta in {4,8}, each uniform; chain c uses field seed 4000 + c."""
    rng = np.random.default_rng(seed)
    Ls = rng.choice([6, 9, 12, 15], size=n_chains)
    Us = rng.choice([-3.0, -4.0, -5.0], size=n_chains)
    betas = rng.choice([4.0, 8.0], size=n_chains)
    out = []
    for c in range(n_chains):
        out.append(Workload(f"chain{c}", L=int(Ls[c]), U=float(Us[c]), beta=float(betas[c]),
                            delay_k=32, sweeps=1, seed=4000 + c, prec="fp32"))
    return out


def ising_fields_n(n_sites: int, L_tau: int, seed: int) -> np.ndarray:
    """i.i.d. +-1 fields for any lattice, shape (L_tau, n_sites), dtype int8."""
    rng = np.random.default_rng(seed)
    return (2 * rng.integers(0, 2, size=(L_tau, n_sites)) - 1).astype(np.int8)


def metropolis_uniforms_n(n_sites: int, L_tau: int, seed: int, n_sweeps: int = 1) -> np.ndarray:
    """U[0,1) draws for any lattice, shape (n_sweeps, L_tau, n_sites), float64."""
    rng = np.random.default_rng(seed + 10**6)
    return rng.random((n_sweeps, L_tau, n_sites))


def ising_fields(L: int, L_tau: int, seed: int) -> np.ndarray:
    """i.i.d. +-1 fields of the kagome lattice, shape (L_tau, 3*L*L), dtype int8."""
    return ising_fields_n(3 * L * L, L_tau, seed)


def metropolis_uniforms(L: int, L_tau: int, seed: int, n_sweeps: int = 1) -> np.ndarray:
    """U[0,1) draws of the kagome lattice, shape (n_sweeps, L_tau, 3*L*L), float64."""
    return metropolis_uniforms_n(3 * L * L, L_tau, seed, n_sweeps)


def random_dense(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """A dense float64 test matrix with entries U(-scale, scale)."""
    rng = np.random.default_rng(seed)
    return scale * (2.0 * rng.random((n, n)) - 1.0)


def l_tau(beta: float, dtau: float) -> int:
    n = int(round(beta / dtau))
    if not math.isclose(n * dtau, beta, rel_tol=1e-9):
        raise ValueError("beta must be a multiple of dtau")
    return n
