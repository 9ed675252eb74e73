"""Named, seeded random streams for the synthetic inputs.

Each (seed, stream name) pair gets its own PCG64 generator, so adding draws to
one stream never shifts another.  Normal variates use the Box-Muller transform
over uniform doubles, which keeps them independent of NumPy's choice of normal
sampler.  The solvers themselves never draw random numbers.
"""
from __future__ import annotations

import hashlib

import numpy as np

STREAMS = {
    "coef": 1,
    "perm": 2,
    "rhs": 3,
    "vel": 4,
    "sizes": 5,
    "target": 6,
    "fd": 7,
    "x0": 8,
    "test": 9,
    "src": 10,
}


def stream(seed: int, name: str) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), STREAMS[name]])))


def normal(rng: np.random.Generator, size) -> np.ndarray:
    """Standard normal variates by Box-Muller (cosine branch)."""
    size = int(size)
    u1 = 1.0 - rng.random(size)  # (0, 1]
    u2 = rng.random(size)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def lognormal(rng: np.random.Generator, size, mu=0.0, sigma=1.0) -> np.ndarray:
    return np.exp(mu + sigma * normal(rng, size))


def uniform(rng: np.random.Generator, size, lo=-1.0, hi=1.0) -> np.ndarray:
    return lo + (hi - lo) * rng.random(int(size))


def sha256(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
