"""FP64 oracle of the hydrogen photoionisation workload -- TEST INFRASTRUCTURE ONLY.

The R-type expansion test of sec. 3.1.1: a point source of Ndot ionising
photons/s in uniform hydrogen of density n_H, one frequency bin, constant
cross section sigma_H and case B recombination coefficient alpha_B (the values
of the tests section).  Each time step:

 1. transport: the sweep under the exponential cell law (see sweep_oracle.c)
    with kappa_c = n_H y_c sigma_H (y: neutral fraction) and the source's
    emission in units of Ndot, giving the photons absorbed per second in every
    cell, Ndot * absorbed_c;
 2. the step length: no cell may gain more ionised atoms (net of its current
    recombinations) than it has neutral atoms,
        dt = min(dt_max, t_left, f * min_c n_H V_c y_c / (Ndot absorbed_c - alpha_B n_H^2 u_c^2 V_c))
    over the cells with a positive denominator (u = 1 - y, f <= 1);
 3. chemistry, photon conserving with implicit recombination: every absorbed
    photon ionises one atom,
        n_H V (u' - u) = Ndot absorbed dt - alpha_B n_H^2 u'^2 V dt,
    i.e. a u'^2 + u' - b = 0 with a = alpha_B n_H dt, b = u + Ndot absorbed dt / (n_H V),
    solved as u' = 2 b / (1 + sqrt(1 + 4 a b)); step 2 keeps u' <= 1.

Only the test-suite may import this module; it shares no code with the GPU
library.  The analytic R-type radius and the Stromgren radius are eq.
rtypeRadius and the Stromgren formula of sec. 3.1.
"""
from __future__ import annotations

import numpy as np

from . import forward


def stromgren_radius(p: dict) -> float:
    """(3 Ndot / (4 pi alpha_B n_H^2))^(1/3), in cm (ionised medium, n_e = n_H+ = n_H)."""
    return (3.0 * p["photon_rate"] / (4.0 * np.pi * p["alpha_B"] * p["n_H"] ** 2)) ** (1.0 / 3.0)


def recombination_time(p: dict) -> float:
    return 1.0 / (p["alpha_B"] * p["n_H"])


def rtype_radius(t: np.ndarray, p: dict) -> np.ndarray:
    """Eq. rtypeRadius: R_St (1 - e^{-t/t_rec})^(1/3)."""
    return stromgren_radius(p) * (1.0 - np.exp(-np.asarray(t) / recombination_time(p))) ** (1.0 / 3.0)


def kappa_of(y: np.ndarray, p: dict) -> np.ndarray:
    """Extinction per mesh length unit: n_H y sigma_H L."""
    return p["n_H"] * y * p["sigma_H"] * p["length_unit"]


def ion_limit(absorbed: np.ndarray, y: np.ndarray, V: np.ndarray, p: dict) -> float:
    """min over cells of n_H V y / (net ionisations per second), +inf if none is positive.
    absorbed in units of Ndot, V in cm^3."""
    u = 1.0 - y
    net = p["photon_rate"] * absorbed - p["alpha_B"] * p["n_H"] ** 2 * u * u * V
    m = net > 0.0
    if not m.any():
        return np.inf
    return float(np.min(p["n_H"] * V[m] * y[m] / net[m]))


def ion_update(absorbed: np.ndarray, y: np.ndarray, V: np.ndarray, dt: float, p: dict) -> np.ndarray:
    """Neutral fraction after a photon-conserving step of length dt."""
    u = 1.0 - y
    a = p["alpha_B"] * p["n_H"] * dt
    b = u + p["photon_rate"] * absorbed * dt / (p["n_H"] * V)
    un = 2.0 * b / (1.0 + np.sqrt(1.0 + 4.0 * a * b))
    return 1.0 - np.minimum(un, 1.0)


def evolve(w: dict, t_end: float, max_steps: int = 1_000_000, record=None, dir_sets=None):
    """Time-step workload `w` (one mesh, G = 1, no scattering, exponential law; w["hii"]
    holds the physical parameters) from a neutral start to t_end seconds.  Returns (t, y) and
    calls record(step, t, y, absorbed, dt) after every step when given.  dir_sets: a list
    of direction sets used in turn, one per step (the rotated directions of sec. 2.6
    that smear out the preferred directions); default w["dirs"] for every step."""
    p = w["hii"]
    (mesh,) = w["meshes"]
    V = np.asarray(mesh["cell_volume"], np.float64) * p["length_unit"] ** 3
    y = np.ones(len(V))
    t = 0.0
    ww = dict(w, law="exp")
    for step in range(max_steps):
        if t >= t_end:
            break
        ww["kappa"] = kappa_of(y, p)[:, None]
        if dir_sets is not None:
            ww["dirs"] = dir_sets[step % len(dir_sets)]
        absorbed = forward(ww)["absorbed"][:, 0]
        dt_max = p["dt_max_trec"] * recombination_time(p)
        dt = min(dt_max, t_end - t, p["courant"] * ion_limit(absorbed, y, V, p))
        y = ion_update(absorbed, y, V, dt, p)
        t += dt
        if record is not None:
            record(step, t, y, absorbed, dt)
    return t, y
