"""Seeded densities and far-field velocities (inputs only; no arithmetic of the method)."""
from __future__ import annotations

import numpy as np


def random_scalar(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).normal(size=n)


def random_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).normal(size=(3, n))


def smooth_scalar(x: np.ndarray, seed: int) -> np.ndarray:
    """A smooth field on the nodes: a random cubic polynomial of the coordinates."""
    rng = np.random.default_rng(seed)
    c = rng.normal(size=10)
    X, Y, Z = x
    return (c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * Y + c[5] * Y * Z + c[6] * Z * X
            + c[7] * X**2 * Y + c[8] * Z**3 + c[9] * X * Y * Z)


def smooth_vector(x: np.ndarray, seed: int) -> np.ndarray:
    return np.stack([smooth_scalar(x, seed + k) for k in range(3)])


def unit_vector(seed: int) -> np.ndarray:
    """A direction drawn uniformly on the unit sphere."""
    v = np.random.default_rng(seed).normal(size=3)
    return v / np.linalg.norm(v)


def point_cloud(n: int, seed: int):
    """Arbitrary node set (not a surface): points, unit normals, positive weights."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(3, n))
    nr = rng.normal(size=(3, n))
    nr /= np.linalg.norm(nr, axis=0)
    w = rng.uniform(0.0, 0.01, size=n)
    return x, nr, w
