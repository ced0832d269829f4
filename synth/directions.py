"""Discrete direction sets (unit vectors, FP64).

Every direction owns the solid angle 4*pi/D (section 2.6 of the paper).  The
paper's 84-direction simulated-annealing table is not available, so:
  * D = 8: the octant diagonals (+-1,+-1,+-1)/sqrt(3), sign order '-' before '+'
    with x varying slowest;
  * any D: a spherical Fibonacci lattice z_k = 1 - (2k+1)/D, phi_k = k*pi*(3-sqrt 5).
"""
from __future__ import annotations

import numpy as np


def octant_diagonals() -> np.ndarray:
    s = 1.0 / np.sqrt(3.0)
    out = []
    for sx in (-1.0, 1.0):
        for sy in (-1.0, 1.0):
            for sz in (-1.0, 1.0):
                out.append((sx * s, sy * s, sz * s))
    return np.array(out, dtype=np.float64)


def fibonacci(D: int) -> np.ndarray:
    k = np.arange(D, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / D
    phi = k * np.pi * (3.0 - np.sqrt(5.0))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    d = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def direction_set(D: int) -> np.ndarray:
    return octant_diagonals() if D == 8 else fibonacci(D)


def rotation(theta: float, phi: float) -> np.ndarray:
    """Rotation by theta about y followed by phi about z."""
    ct, st, cp, sp = np.cos(theta), np.sin(theta), np.cos(phi), np.sin(phi)
    ry = np.array([[ct, 0.0, st], [0.0, 1.0, 0.0], [-st, 0.0, ct]])
    rz = np.array([[cp, -sp, 0.0], [sp, cp, 0.0], [0.0, 0.0, 1.0]])
    return rz @ ry


def rotated_sets(D: int, n_rot: int, seed: int = 0) -> list:
    """n_rot copies of direction_set(D), each rotated by seeded random angles
    theta in [0, pi], phi in [0, 2 pi] (the first copy unrotated), renormalised."""
    rng = np.random.default_rng(np.random.SeedSequence([2207, 12848, 7, seed]))
    base = direction_set(D)
    out = [base]
    for _ in range(n_rot - 1):
        r = rotation(rng.uniform(0.0, np.pi), rng.uniform(0.0, 2.0 * np.pi))
        d = base @ r.T
        out.append(d / np.linalg.norm(d, axis=1, keepdims=True))
    return out
