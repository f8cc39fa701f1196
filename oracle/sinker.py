"""Multi-sinker viscosity and body force (paper Sec. 2.1, the benchmark definition).

TEST INFRASTRUCTURE ONLY (see the package header).

Pinned by: mu = mu_max at every centre, mu in [mu_min, mu_max], no sinkers
gives mu = mu_min everywhere (tests/test_oracle_basics.py).
"""
from __future__ import annotations

import numpy as np


def chi(x: np.ndarray, centers: np.ndarray, delta: float, omega: float) -> np.ndarray:
    """Indicator chi_n(x): product over sinkers of 1 - exp(-delta max(0, |c_i - x| - omega/2)^2).

    x: [..., 3] points.  Returns [...]."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones(x.shape[:-1])
    for c in np.asarray(centers, dtype=np.float64).reshape(-1, 3):
        dist = np.sqrt(np.sum((x - c) ** 2, axis=-1))
        s = np.maximum(0.0, dist - 0.5 * omega)
        out = out * (1.0 - np.exp(-delta * s * s))
    return out


def viscosity(x, centers, delta, omega, mu_min, mu_max):
    """mu(x) = (mu_max - mu_min)(1 - chi_n(x)) + mu_min."""
    return (mu_max - mu_min) * (1.0 - chi(x, centers, delta, omega)) + mu_min


def body_force(x, centers, delta, omega, beta=10.0):
    """f(x) = (0, 0, beta (chi_n(x) - 1)); returns [..., 3]."""
    c = chi(x, centers, delta, omega)
    f = np.zeros(np.shape(c) + (3,))
    f[..., 2] = beta * (c - 1.0)
    return f
