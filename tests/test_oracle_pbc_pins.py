"""Pins of the oracle's merged periodic/scattering iterations and warm start (sec.
2.7's periodic passes and algorithm 1's source iteration run as one sequence,
and the periodic inflow of the first pass taken from an earlier solution): the
dense fixed point of the coupled cyclic + scattering system, the cost advantage
over the nested order, identity where the orders coincide, conservation, and the
warm start's fixed-point property."""
import numpy as np

import oracle
from synth import workloads as W
from tests import dense_reference as DR


def _w(**kw):
    return W.small_random(180, 8, G=1, seed=3, periodic=True, n_src=3, tau=2.0, albedo=0.6, **kw)


def _err(r, Jfix):
    return np.max(np.abs(r["J"][:, 0] - Jfix) / Jfix)


def test_merged_and_nested_reach_the_dense_fixed_point():
    w = _w()
    Jfix = DR.dense_scatter_system(w, cyclic=True).sum(0) / (4 * np.pi)
    m = oracle.forward(dict(w, n_pbc=300, n_scat=300, merge=True))
    n = oracle.forward(dict(w, n_pbc=60, n_scat=60))
    assert _err(m, Jfix) < 1e-12
    assert _err(n, Jfix) < 1e-10


def test_merged_is_cheaper_at_equal_pass_count():
    """64 merged passes against 8 source iterations of 8 periodic passes each."""
    w = _w()
    Jfix = DR.dense_scatter_system(w, cyclic=True).sum(0) / (4 * np.pi)
    m = _err(oracle.forward(dict(w, n_pbc=64, n_scat=64, merge=True)), Jfix)
    n = _err(oracle.forward(dict(w, n_pbc=8, n_scat=8)), Jfix)
    assert m < 1e-3 * n


def test_merged_equals_nested_where_the_orders_coincide():
    for w in (_w(n_pbc=5, n_scat=1), dict(_w(n_pbc=1, n_scat=4), boundary="vacuum",
                                          meshes=[W.small_random(180, 8, seed=3)["meshes"][0]])):
        a = oracle.forward(dict(w, merge=True), want_phi=True)
        b = oracle.forward(w, want_phi=True)
        assert np.array_equal(a["J"], b["J"]) and np.array_equal(a["phi"][0], b["phi"][0])
        assert np.array_equal(a["totals"], b["totals"])


def test_merged_conserves_photons():
    w = dict(_w(n_pbc=3, n_scat=7), merge=True)
    for law in ("upwind", "exp"):
        t = oracle.forward(dict(w, law=law))["totals"][0]
        lhs = t[:, 0] + t[:, 3] + t[:, 5]
        rhs = t[:, 1] + t[:, 2] + t[:, 4]
        assert np.all(np.abs(lhs - rhs) <= 1e-12 * t[:, 0])


def test_warm_start_from_the_fixed_point_stays_there():
    w = _w(n_scat=1)
    conv = oracle.forward(dict(w, n_pbc=300), want_phi=True)
    one = oracle.forward(dict(w, n_pbc=1), want_phi=True, phi_init=conv["phi"])
    assert np.max(np.abs(one["J"] - conv["J"]) / conv["J"]) < 1e-12
    # without the warm start one pass is far from it
    cold = oracle.forward(dict(w, n_pbc=1))
    assert np.max(np.abs(cold["J"] - conv["J"]) / conv["J"]) > 1e-2


def test_warm_start_continues_the_passes():
    """k passes, then m passes warm-started from the k-th pass's phi, equal k + m passes."""
    w = _w(n_scat=1)
    a = oracle.forward(dict(w, n_pbc=3), want_phi=True)
    b = oracle.forward(dict(w, n_pbc=4), want_phi=True, phi_init=a["phi"])
    c = oracle.forward(dict(w, n_pbc=7), want_phi=True)
    assert np.allclose(b["J"], c["J"], rtol=1e-13, atol=0)
    assert np.allclose(b["phi"][0], c["phi"][0], rtol=1e-13, atol=1e-300)


def test_convergence_threshold_stops_the_passes():
    """pbc_tol (sec. 2.7): the passes stop at the first pass k >= 2 whose E is below the
    threshold in every cell; the result is then exactly that of k passes."""
    w = _w(n_scat=1)
    emax = [oracle.forward(dict(w, n_pbc=n))["totals"][0, :, 6].max() for n in range(2, 12)]
    tol = 0.5 * (emax[4] + emax[5])  # between the E of 6 and of 7 passes
    k = 2 + next(i for i, e in enumerate(emax) if e < tol)
    assert k == 7
    r = oracle.forward(dict(w, n_pbc=40, pbc_tol=tol), want_phi=True)
    ref = oracle.forward(dict(w, n_pbc=k), want_phi=True)
    assert np.array_equal(r["J"], ref["J"]) and np.array_equal(r["phi"][0], ref["phi"][0])
    assert np.array_equal(r["totals"], ref["totals"])
    assert r["totals"][0, :, 6].max() < tol
    # a threshold no pass reaches runs all n_pbc passes
    r = oracle.forward(dict(w, n_pbc=5, pbc_tol=1e-30))
    assert np.array_equal(r["J"], oracle.forward(dict(w, n_pbc=5))["J"])
