"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds random draws only: no transform, no operator, no grid and
no arithmetic of the spectral method.  Each side turns these draws into its
own initial condition with its own grid and its own code.

Rayleigh-Benard workloads (2-D and 3-D) perturb the conductive buoyancy
profile with unit-variance Gaussian noise on the scale-1 grid; the noise array
is drawn once with NumPy's PCG64 generator and handed to both sides unchanged.
"""
from __future__ import annotations

import numpy as np

# Seed convention: workload number c uses seed 1000 + c; finite-difference
# directions for the adjoint use 2000 + r.
WORKLOAD_SEED_BASE = 1000
DIRECTION_SEED_BASE = 2000


def noise(shape, seed: int) -> np.ndarray:
    """Standard-normal float64 array of `shape` (C order) from PCG64(seed)."""
    return np.random.default_rng(seed).standard_normal(tuple(int(s) for s in shape))


def workload_noise(shape, workload: int) -> np.ndarray:
    return noise(shape, WORKLOAD_SEED_BASE + int(workload))


def direction(shape, r: int) -> np.ndarray:
    """Unit-norm random direction number r (for directional derivatives)."""
    d = noise(shape, DIRECTION_SEED_BASE + int(r))
    return d / np.linalg.norm(d)


def complex_noise(shape, seed: int) -> np.ndarray:
    """Complex128 array whose real and imaginary parts are independent N(0,1)."""
    g = np.random.default_rng(seed)
    s = tuple(int(x) for x in shape)
    return g.standard_normal(s) + 1j * g.standard_normal(s)
