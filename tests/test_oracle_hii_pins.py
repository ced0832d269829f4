"""Pins of the photoionisation oracle (R-type expansion of sec. 3.1.1): the
chemistry step against photon counting, ionisation equilibrium and the closed
form of pure recombination; the coupled sweep + chemistry evolution against the
analytic R-type radius (eq. rtypeRadius) and the Stromgren sphere."""
import numpy as np

from oracle import hii as H
from synth import workloads as W
from tests import hii_analysis as HA


def _params():
    return W.hii_rtype(4, 8)["hii"]


def test_paper_radius_and_recombination_time():
    """The tests section quotes R_St = 6.79 kpc and t_rec = 122.4 Myr for these parameters."""
    p = _params()
    assert abs(H.stromgren_radius(p) / W.KPC_CM - 6.79) < 0.01
    assert abs(H.recombination_time(p) / 3.15576e13 - 122.4) < 0.1


def test_ion_update_conserves_photons_and_keeps_equilibrium():
    p = _params()
    rng = np.random.default_rng(1)
    C = 500
    V = rng.uniform(0.5, 2.0, C) * 1e63
    y = rng.uniform(0.0, 1.0, C)
    ab = rng.uniform(0.0, 1e-3, C)
    dt = 0.9 * H.ion_limit(ab, y, V, p)
    yn = H.ion_update(ab, y, V, dt, p)
    u, un = 1 - y, 1 - yn
    assert np.all(un <= 1.0) and np.all(un >= 0.0)
    # every absorbed photon ionises one atom, net of recombinations at the new state
    lhs = p["n_H"] * V * (un - u) + p["alpha_B"] * p["n_H"] ** 2 * un ** 2 * V * dt
    rhs = p["photon_rate"] * ab * dt
    assert np.allclose(lhs, rhs, rtol=1e-9, atol=1e-12 * rhs.max())
    # photoionisation balancing recombination leaves the state unchanged
    ab_eq = p["alpha_B"] * p["n_H"] ** 2 * u ** 2 * V / p["photon_rate"]
    ye = H.ion_update(ab_eq, y, V, 0.3 * H.recombination_time(p), p)
    assert np.allclose(1 - ye, u, rtol=1e-12, atol=1e-15)


def test_pure_recombination_converges_to_closed_form():
    """No radiation: du/dt = -alpha n u^2 from u = 1 gives u = 1 / (1 + t / t_rec); the
    implicit steps converge to it at first order."""
    p = _params()
    V = np.ones(1)
    T = 2.0 * H.recombination_time(p)
    exact = 1.0 / (1.0 + 2.0)
    errs = []
    for n in (50, 100, 200):
        y = np.zeros(1)
        for _ in range(n):
            y = H.ion_update(np.zeros(1), y, V, T / n, p)
        errs.append(abs((1 - y[0]) - exact))
    assert errs[0] > errs[1] > errs[2]
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


def _run(w, t_end_trec, every=1):
    p = w["hii"]
    mesh = w["meshes"][0]
    V = mesh["cell_volume"] * p["length_unit"] ** 3
    r = HA.cell_radius(mesh, w["source_pos"], p["length_unit"])
    trec = H.recombination_time(p)
    rows = []

    def rec(step, t, y, ab, dt):
        if step % every == 0:
            rows.append((t / trec, HA.volume_radius(y, V), HA.half_ionised_radius(y, r, p["length_unit"] / 16),
                         np.sum(p["alpha_B"] * p["n_H"] ** 2 * (1 - y) ** 2 * V), dt))
    H.evolve(w, t_end_trec * trec, record=rec)
    return np.array(rows)


def test_rtype_expansion_follows_the_analytic_radius():
    w = W.hii_rtype(16, 24)
    p = w["hii"]
    rows = _run(w, 1.5)
    t, rv, rh = rows[:, 0], rows[:, 1], rows[:, 2]
    ra = H.rtype_radius(t * H.recombination_time(p), p)
    late = t >= 0.05
    # the volume radius follows eq. rtypeRadius within 5 % at 16^3 and 24 directions
    assert np.all(np.abs(rv[late] / ra[late] - 1) < 0.05)
    assert np.all(np.abs(rh[t >= 0.25] / ra[t >= 0.25] - 1) < 0.1)
    assert np.all(np.diff(rv) >= -1e-9 * rv[1:])  # the front never recedes


def test_stromgren_sphere_is_reached():
    """A ten times weaker source: after 5 recombination times the sphere is in
    equilibrium: its half-ionised radius is R_St and the recombinations balance
    the emitted photons.  (The volume radius is larger by the partly ionised
    cells of the front, a few per cent at 4 cells per R_St.)"""
    w = W.hii_rtype(16, 24)
    p = w["hii"]
    p["photon_rate"] = 1e48
    rows = _run(w, 5.0)
    rs = H.stromgren_radius(p)
    assert abs(rows[-1, 2] / rs - 1) < 0.03
    assert 1.0 < rows[-1, 1] / rs < 1.1
    assert abs(rows[-1, 3] / p["photon_rate"] - 1) < 0.05


def test_direction_sets_in_turn():
    """Cycling identical direction sets changes nothing; a set turned by 90 degrees
    about z through the source's cell turns the ionisation field with it (before the
    front reaches the box walls, which sit half a cell off-centre)."""
    from synth.directions import rotation
    w = W.hii_rtype(16, 24)
    p = w["hii"]
    t_end = 0.05 * H.recombination_time(p)
    _, y1 = H.evolve(w, t_end)
    _, y2 = H.evolve(w, t_end, dir_sets=[w["dirs"], w["dirs"].copy()])
    assert np.array_equal(y1, y2)
    rz = rotation(0.0, 0.5 * np.pi)
    _, yr = H.evolve(w, t_end, dir_sets=[w["dirs"] @ rz.T])
    n, c = 16, 8
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    # the cell at offset (x, y) from the source's cell maps to offset (-y, x)
    ii, jj = c - (j - c), c + (i - c)
    ok = (ii >= 0) & (ii < n) & (jj >= 0) & (jj < n)
    src = (i + n * (j + n * k))[ok]
    dst = (ii + n * (jj + n * k))[ok]
    assert np.max(np.abs(yr[dst] - y1[src])) < 1e-9


def test_rotated_sets_reduce_the_radius_error():
    """Five rotated sets in turn (sec. 2.6's N_rot = 5) against one fixed set."""
    from synth.directions import rotated_sets
    w = W.hii_rtype(16, 24)
    p = w["hii"]
    t_end = 0.5 * H.recombination_time(p)
    V = w["meshes"][0]["cell_volume"] * p["length_unit"] ** 3
    ra = H.rtype_radius(t_end, p)
    errs = []
    for n_rot in (1, 5):
        _, y = H.evolve(w, t_end, dir_sets=rotated_sets(24, n_rot))
        errs.append(abs(HA.volume_radius(y, V) / ra - 1))
    assert errs[1] < errs[0] < 0.02
