"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the method: it only names the workload
configurations and draws seeded random numbers (sinker centres, test vectors).
Both the GPU library and the CPU oracle receive these arrays as inputs.

Workloads follow the multi-sinker benchmark of the paper (Sec. 2.1): the unit
cube, n sinkers at random centres, decay delta, diameter omega, dynamic ratio
DR with mu_min = DR^-1/2 and mu_max = DR^1/2, body-force scale beta = 10.
The paper's own centres are not published, so centres are drawn from
``numpy.random.default_rng(seed).random((n, 3))``.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    N: int            # elements per direction
    k: int            # velocity order (pressure order k-1)
    n_sinkers: int
    delta: float
    omega: float
    dr: float         # dynamic ratio mu_max / mu_min
    a_l: float        # left boundary amplification (Sec. 5)
    a_r: float        # right boundary amplification (Sec. 5)
    seed: int
    beta: float = 10.0

    @property
    def mu_min(self) -> float:
        return self.dr ** -0.5

    @property
    def mu_max(self) -> float:
        return self.dr ** 0.5

    def centers(self) -> np.ndarray:
        return sinker_centers(self.seed, self.n_sinkers)

    @property
    def n_nodes(self) -> int:
        return (self.k * self.N + 1) ** 3

    @property
    def u_dof(self) -> int:
        return 3 * self.n_nodes

    @property
    def p_dof(self) -> int:
        return self.N ** 3 * self.k * (self.k + 1) * (self.k + 2) // 6

    def describe(self) -> str:
        return (f"{self.name}: {self.N}^3 elements, Q{self.k} x P{self.k - 1}-disc, {self.n_sinkers} "
                f"seeded sinkers, delta {self.delta:g}, omega {self.omega:g}, DR {self.dr:g}, "
                f"a_r {self.a_r:g}, FGMRES(100) to 1e-6")


def default_a_r(N: int, k: int) -> float:
    """Right boundary amplification schedule max(1, (N/16) * 2^(k-2)).

    Reproduces every a_r entry of the paper's Table 3 (a_l = 1 there)."""
    return float(max(1.0, (N / 16.0) * 2.0 ** (k - 2)))


# The five workloads: 4^3 Q2 (small, oracle-sized), 32^3 Q2, 16^3 Q4,
# 48^3 Q2 (learned coarse correction) and 64^3 Q3 (largest).
WORKLOADS = {
    "c1": Workload("c1", 4, 2, 4, 200.0, 0.1, 1e4, 1.0, default_a_r(4, 2), 1),
    "c2": Workload("c2", 32, 2, 16, 200.0, 0.1, 1e6, 1.0, default_a_r(32, 2), 2),
    "c3": Workload("c3", 16, 4, 24, 200.0, 0.05, 1e8, 1.0, default_a_r(16, 4), 3),
    "c4": Workload("c4", 48, 2, 32, 200.0, 0.1, 1e10, 1.0, default_a_r(48, 2), 4),
    "c5": Workload("c5", 64, 3, 48, 300.0, 0.04, 1e10, 1.0, default_a_r(64, 3), 5),
}


def custom(name: str, N: int, k: int, n_sinkers: int = 4, delta: float = 200.0,
           omega: float = 0.1, dr: float = 1e4, a_l: float = 1.0,
           a_r: float | None = None, seed: int = 0) -> Workload:
    return Workload(name, N, k, n_sinkers, delta, omega, dr, a_l,
                    default_a_r(N, k) if a_r is None else a_r, seed)


def sinker_centers(seed: int, n: int) -> np.ndarray:
    """Sinker centres, uniform in the unit cube, shape [n, 3], float64."""
    return np.random.default_rng(seed).random((n, 3))


def random_vector(seed: int, size: int) -> np.ndarray:
    """Uniform [-1, 1) test vector, float64."""
    return np.random.default_rng(seed + 7919).uniform(-1.0, 1.0, size)


# Learned coarse correction: training fields from seeds 1000..2999 and validation fields from
# seeds 3000..3099 (disjoint from the evaluation seeds 1..5), each with the workload's sinker count.
TRAIN_SEEDS = range(1000, 3000)
VALID_SEEDS = range(3000, 3100)


def learned_fields(w: Workload, n_train: int = len(TRAIN_SEEDS), n_valid: int = len(VALID_SEEDS)):
    """Sinker centres of the training and validation fields of workload w."""
    train = [sinker_centers(s, w.n_sinkers) for s in list(TRAIN_SEEDS)[:n_train]]
    valid = [sinker_centers(s, w.n_sinkers) for s in list(VALID_SEEDS)[:n_valid]]
    return train, valid
