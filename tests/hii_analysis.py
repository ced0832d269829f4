"""Radius of an ionised region on a lattice (analysis helper of the HII tests).

Two definitions: the equivalent-volume radius (3 sum u V / 4 pi)^(1/3) of the
ionised fraction u = 1 - y, and the radius of sec. 3.1.1 at which the average
ionised fraction over a spherical shell falls to 0.5 (shells of one cell
width around the source, linear interpolation between shell centres).
"""
from __future__ import annotations

import numpy as np


def cell_radius(mesh: dict, src_pos, length_unit: float) -> np.ndarray:
    return np.linalg.norm(np.asarray(mesh["points"]) - np.asarray(src_pos)[None, :], axis=1) * length_unit


def volume_radius(y: np.ndarray, V: np.ndarray) -> float:
    return float((3.0 * np.sum((1.0 - y) * V) / (4.0 * np.pi)) ** (1.0 / 3.0))


def half_ionised_radius(y: np.ndarray, r: np.ndarray, width: float) -> float:
    u = 1.0 - np.asarray(y)
    k = np.floor(r / width).astype(np.int64)
    n = np.bincount(k)
    s = np.bincount(k, weights=u)
    ok = n > 0
    centres = (np.arange(len(n)) + 0.5)[ok] * width
    avg = s[ok] / n[ok]
    below = np.nonzero(avg < 0.5)[0]
    if len(below) == 0:
        return float(centres[-1])
    i = below[0]
    if i == 0:
        return float(centres[0] * avg[0] / 0.5)
    a0, a1 = avg[i - 1], avg[i]
    return float(centres[i - 1] + (a0 - 0.5) / (a0 - a1) * (centres[i] - centres[i - 1]))
