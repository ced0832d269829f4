"""Pins of the oracle's exponential cell law (transmission e^{-tau} through a cell
of optical depth tau = kappa V / Aperp, the attenuation form 1 - e^{-dn sigma} of
the scattering test of sec. 3.3 with the mean chord V / Aperp as the distance
travelled): exact attenuation of aligned beams, a one-cell closed form, the
kappa = 0 limit where it must coincide with the upwind balance, conservation,
dense solves of the same linear systems, and central differences of the adjoint."""
import numpy as np
import pytest

import oracle
from synth import workloads as W
from synth.directions import direction_set
from tests import dense_reference as DR


def _rel(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def _exp(w):
    return dict(w, law="exp")


# ----------------------------------------------------------------------------- closed forms
@pytest.mark.parametrize("kappa", [0.5, 3.0])
def test_exp_aligned_beam_is_exact_exponential(kappa):
    """Omega = +x on an n^3 lattice: every cell of width h multiplies the beam by
    exactly e^{-kappa h}, so the slab transmits exactly e^{-kappa} (the analytic
    attenuation, with no first-order error)."""
    n = 8
    h = 1.0 / n
    row = [m + n * (3 + n * 5) for m in range(n)]
    w = _exp(W.lattice_workload(n, np.array([[1.0, 0.0, 0.0]]), kappa, [row[0]], [2.0]))
    r = oracle.forward(w, want_phi=True)
    kap = float(w["kappa"][0, 0])  # inputs are rounded to FP32 once
    m = np.arange(n)
    # exit flux density: power 2 e^{-kappa h (m+1)} through the exit face of area h^2
    x = r["phi"][0][0, :, 0]
    assert _rel(x[row], 2.0 * np.exp(-kap * h * (m + 1)) / h ** 2) < 1e-13
    # cell average: absorbed power / (kappa V), absorbed = 2 e^{-kappa h m} (1 - e^{-kappa h})
    avg = 2.0 * np.exp(-kap * h * m) * (1.0 - np.exp(-kap * h)) / (kap * h ** 3)
    assert _rel(r["J"][row, 0], avg / (4 * np.pi)) < 1e-13
    mask = np.ones(n ** 3, bool)
    mask[row] = False
    assert np.all(x[mask] == 0.0) and np.all(r["J"][mask] == 0.0)
    t = r["totals"][0, 0]
    assert abs(t[2] - 2.0 * np.exp(-kap)) < 1e-14 * 2.0  # escaped = L e^{-kappa L}
    assert abs(t[1] - 2.0 * (1.0 - np.exp(-kap))) < 1e-14 * 2.0


def test_exp_single_cell_closed_form():
    """Unit cube, D directions: Aperp_d = |Ox|+|Oy|+|Oz|, V = 1, so direction d
    transmits (L/D) e^{-kappa/Aperp_d} and its cell average is
    (L/D)(1 - e^{-kappa/Aperp_d}) / kappa."""
    dirs = direction_set(24)
    w = _exp(W.lattice_workload(1, dirs, 0.7, [0], [3.0]))
    r = oracle.forward(w, want_phi=True)
    ap = np.abs(dirs).sum(axis=1)
    kap = float(w["kappa"][0, 0])
    trans = (3.0 / 24) * np.exp(-kap / ap)
    assert _rel(r["phi"][0][:, 0, 0], trans / ap) < 1e-14
    avg = (3.0 / 24) * (1.0 - np.exp(-kap / ap)) / kap
    assert _rel(r["J"][0, 0], avg.sum() / (4 * np.pi)) < 1e-14
    assert _rel(r["totals"][0, 0, 2], trans.sum()) < 1e-14


def test_exp_equals_upwind_without_absorption():
    """kappa = 0: no attenuation in either law, both give phi = T / Aperp bit for bit."""
    w = W.small_random(300, 24, G=2, seed=21, n_src=5, n_meshes=2)
    w["kappa"] = np.zeros_like(w["kappa"])
    a = oracle.forward(w, want_phi=True)
    b = oracle.forward(_exp(w), want_phi=True)
    for x, y in zip(a["phi"], b["phi"]):
        assert np.array_equal(x, y)
    assert np.array_equal(a["J"], b["J"]) and np.array_equal(a["totals"], b["totals"])


def test_exp_differs_from_upwind_at_second_order():
    """Thin cells: per cell the upwind law passes on 1/(1+tau), the exponential
    law e^{-tau}; the exit flux densities differ at O(tau^2) relative."""
    n = 8
    h = 1.0 / n
    row = [m + n * (3 + n * 5) for m in range(n)]
    for kappa in (0.08, 0.04):
        w = W.lattice_workload(n, np.array([[1.0, 0.0, 0.0]]), kappa, [row[0]], [1.0])
        up = oracle.forward(w, want_phi=True)["phi"][0][0, row, 0]
        ex = oracle.forward(_exp(w), want_phi=True)["phi"][0][0, row, 0]
        tau = float(w["kappa"][0, 0]) * h
        # ratio per cell e^{-tau}(1+tau) = 1 - tau^2/2 + O(tau^3)
        ratio = (ex[1:] / ex[:-1]) / (up[1:] / up[:-1])
        assert np.allclose(ratio, np.exp(-tau) * (1 + tau), rtol=1e-13)
        assert np.all(np.abs(ratio - 1 + tau ** 2 / 2) < tau ** 3)


# ----------------------------------------------------------------------------- conservation
def test_exp_conservation_and_thick_limit():
    w = _exp(W.small_random(600, 24, G=3, seed=26, n_src=5, n_meshes=2))
    t = oracle.forward(w)["totals"]
    assert np.all(np.abs(t[..., 0] - t[..., 1] - t[..., 2]) <= 1e-13 * t[..., 0])
    # optical depths far beyond the cap: every photon is absorbed where it is emitted
    wbig = dict(w, kappa=np.full_like(w["kappa"], 1e9))
    rb = oracle.forward(wbig)
    em = np.asarray(w["emission"], np.float64)
    assert np.allclose(rb["absorbed"], em, rtol=1e-15, atol=1e-15 * em.max())
    tb = rb["totals"]
    assert np.all(tb[..., 2] <= 5e-18 * tb[..., 0])  # e^{-40} per cell at most
    assert np.all(np.abs(tb[..., 0] - tb[..., 1] - tb[..., 2]) <= 1e-13 * tb[..., 0])


def test_exp_conservation_with_scattering_and_periodic_passes():
    w = _exp(W.small_random(400, 8, G=2, seed=27, periodic=True, n_src=3, albedo=0.5, n_scat=4,
                            n_pbc=3))
    t = oracle.forward(w)["totals"][0]
    lhs = t[:, 0] + t[:, 3] + t[:, 5]
    rhs = t[:, 1] + t[:, 2] + t[:, 4]
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * t[:, 0])


# ----------------------------------------------------------------------------- dense solves
def test_exp_forward_matches_dense_solve():
    w = _exp(W.small_random(150, 8, G=2, seed=22, n_src=4, tau=4.0))
    r = oracle.forward(w, want_phi=True)
    ref = DR.dense_forward(w)
    assert _rel(r["phi"][0], ref["phi"][0]) < 1e-12
    assert _rel(r["J"], ref["J"]) < 1e-12
    assert _rel(r["absorbed"], ref["absorbed"]) < 1e-12
    assert _rel(r["totals"][..., :3], ref["totals"]) < 1e-12


def test_exp_periodic_passes_converge_to_cyclic_dense_solve():
    w = _exp(W.small_random(180, 8, G=1, seed=3, periodic=True, n_src=3, tau=2.0))
    ref = DR.dense_forward(w, cyclic=True)
    w["n_pbc"] = 200
    r = oracle.forward(w)
    assert _rel(r["J"], ref["J"]) < 1e-10
    t = r["totals"][0, 0]
    assert abs(t[3] - t[4]) / t[4] < 1e-10


def test_exp_scattering_converges_to_dense_system():
    w = _exp(W.small_random(100, 8, G=1, seed=24, n_src=2, albedo=0.5, n_scat=60))
    avg_fix = DR.dense_scatter_system(w)
    r = oracle.forward(w)
    assert _rel(r["J"][:, 0], avg_fix.sum(0) / (4 * np.pi)) < 1e-10


# ----------------------------------------------------------------------------- adjoint
def _loss(w, kind):
    r = oracle.forward(w)
    return r["absorbed"].sum() / (4 * np.pi) if kind == "absorbed" else r["J"].sum()


def _fd_check(w, cells, kind="absorbed", h=1e-6):
    if kind == "absorbed":
        gJ, gA = oracle.absorbed_loss_grads(w)
    else:
        gJ, gA = np.ones_like(w["kappa"]), np.zeros_like(w["kappa"])
    dk, de = oracle.adjoint(w, gJ, gA)
    L = _loss(w, kind)
    for c in cells:
        k0 = w["kappa"][c, 0]
        wp = dict(w, kappa=w["kappa"].copy())
        wm = dict(w, kappa=w["kappa"].copy())
        wp["kappa"][c, 0] = k0 * (1 + h)
        wm["kappa"][c, 0] = k0 * (1 - h)
        fd = (_loss(wp, kind) - _loss(wm, kind)) / (2 * h * k0)
        assert abs(fd - dk[c, 0]) <= 1e-6 * abs(dk[c, 0]) + 1e-10 * L / k0, c
    for c in w["sources"]:
        L0 = w["emission"][c, 0]
        wp = dict(w, emission=w["emission"].copy())
        wm = dict(w, emission=w["emission"].copy())
        wp["emission"][c, 0] = L0 * (1 + h)
        wm["emission"][c, 0] = L0 * (1 - h)
        fd = (_loss(wp, kind) - _loss(wm, kind)) / (2 * h * L0)
        assert abs(fd - de[c, 0]) <= 1e-6 * abs(de[c, 0]), c
    if kind == "absorbed":  # each emitted photon is absorbed at most once
        assert np.all(de >= 0) and np.all(de <= 1 / (4 * np.pi) * (1 + 1e-12))
    return dk, de


@pytest.mark.parametrize("albedo,n_scat", [(0.0, 1), (0.5, 5)])
def test_exp_adjoint_central_differences(albedo, n_scat):
    w = _exp(W.small_random(200, 8, G=1, seed=25, n_src=3, albedo=albedo, n_scat=n_scat))
    w["kappa"] = np.asarray(w["kappa"], np.float64)
    w["emission"] = np.asarray(w["emission"], np.float64)
    rng = np.random.default_rng(2)
    _fd_check(w, rng.choice(200, 8, replace=False))


@pytest.mark.parametrize("kind", ["absorbed", "J"])
def test_exp_adjoint_thin_and_capped_cells(kind):
    """Cells with tau near 0 (series branch of h') and beyond the cap of 40.
    With the absorbed-power loss a capped cell's kappa has no effect (all it
    receives is absorbed, and it passes on the fixed e^{-40}); with L = sum J
    its own J = T (1 - e^{-40}) / (kappa V) gives dL/dkappa = -J / kappa."""
    w = _exp(W.small_random(200, 8, G=1, seed=28, n_src=3, albedo=0.3, n_scat=3))
    w["kappa"] = np.asarray(w["kappa"], np.float64)
    w["emission"] = np.asarray(w["emission"], np.float64)
    rng = np.random.default_rng(3)
    thin = rng.choice(200, 4, replace=False)
    thick = rng.choice(np.setdiff1d(np.arange(200), thin), 4, replace=False)
    V = w["meshes"][0]["cell_volume"]
    w["kappa"][thin, 0] = 3e-2  # tau ~ 3e-3
    w["kappa"][thick, 0] = 400.0 / V[thick] ** (1.0 / 3.0)  # tau of order 100 in every direction
    dk, _ = _fd_check(w, np.concatenate([thin, thick]), kind=kind, h=1e-3)
    if kind == "J":
        J = oracle.forward(w)["J"][:, 0]
        lit = thick[J[thick] > 0]
        assert len(lit) > 0
        assert np.allclose(dk[lit, 0], -J[lit] / w["kappa"][lit, 0], rtol=1e-9)


def test_exp_adjoint_sign_for_mean_intensity_loss():
    """Raising kappa lowers the exit flux and hence every downwind J; in the cell
    itself J = T (1 - e^{-tau}) / (kappa V) also falls with kappa: dL/dkappa <= 0."""
    w = _exp(W.small_random(200, 24, G=1, seed=29, n_src=3))
    dk, _ = oracle.adjoint(w, np.ones((200, 1)), np.zeros((200, 1)))
    assert np.all(dk <= 0)
