"""Pins of the oracle's transport scheme (b) of sec. 2.6 (direction-conserving
transport): a cell's outflow is shared equally by the n = 3 outflow faces whose
normals are the most aligned with the direction, so each task has at most three
downwind dependencies.

- the dense direct solve of the (b) system, assembled from the sending side in
  numpy with no graph (vacuum, the cyclic periodic fixed point, the adjoint);
- levels against brute-force relaxation over the (b) edges;
- a cubic lattice swept along a diagonal, where every cell has exactly three
  outflow faces of equal weight, so (b) and (a) are the same system;
- photon conservation, and at most n_aligned downwind edges per task (so the
  mean in-degree is at most 3, against about 7.8 for scheme (a));
- central differences of the adjoint."""
import numpy as np
import pytest

import oracle
from synth import workloads as W
from synth.mesh import lattice_mesh
from tests import dense_reference as DR


def _w(n=150, D=12, seed=51, **kw):
    return dict(W.small_random(n, D, seed=seed, **kw), scheme="aligned")


def _rel(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300 + 1e-14 * np.abs(b).max()))


@pytest.mark.parametrize("law", ["upwind", "exp"])
def test_aligned_forward_matches_dense_solve(law):
    w = dict(_w(), law=law)
    r = oracle.forward(w)
    d = DR.dense_forward(w)
    assert _rel(r["J"], d["J"]) < 1e-12
    assert _rel(r["absorbed"], d["absorbed"]) < 1e-12
    assert np.allclose(r["totals"][..., :3], d["totals"], rtol=1e-12, atol=0)
    # and it is a different discretisation from scheme (a)
    a = oracle.forward(dict(w, scheme="area"))
    assert _rel(r["J"], a["J"]) > 1e-3


def test_aligned_multimesh_many_faces():
    for w in (_w(120, 8, seed=52, n_meshes=3), dict(W.many_faces(40, 12, seed=4), scheme="aligned")):
        r = oracle.forward(w)
        d = DR.dense_forward(w)
        assert _rel(r["J"], d["J"]) < 1e-12


def test_aligned_periodic_passes_converge_to_cyclic_solve():
    w = _w(160, 8, seed=53, periodic=True, tau=2.0)
    fix = DR.dense_forward(w, cyclic=True)["J"]
    r = oracle.forward(dict(w, n_pbc=200))
    assert _rel(r["J"], fix) < 1e-10
    r3 = oracle.forward(dict(w, n_pbc=3))
    assert np.all(r3["J"] <= fix * (1 + 1e-12))


def test_aligned_levels_match_brute_force_and_are_thin():
    w = _w(300, 16, seed=54)
    mesh = w["meshes"][0]
    lv, od, ind, dep = oracle.build_dag(mesh, w["dirs"], scheme="aligned")
    la, _, inda, _ = oracle.build_dag(mesh, w["dirs"])
    for d in range(len(w["dirs"])):
        bl, src, dst = DR.brute_levels(mesh, w["dirs"][d], scheme="aligned")
        assert np.array_equal(lv[d], bl)
        assert np.array_equal(ind[d], np.bincount(dst, minlength=len(bl)))
        assert np.bincount(src, minlength=len(bl)).max() <= 3
    assert ind.mean() <= 3.0 < inda.mean()


def test_diagonal_lattice_equals_scheme_a():
    """Along (1,1,1)/sqrt(3) every cell of a cubic lattice has three outflow faces
    of equal area and equal Omega . n: scheme (a) already shares the outflow
    equally over exactly those three."""
    n = 6
    mesh = lattice_mesh(n)
    C = n ** 3
    rng = np.random.default_rng(np.random.SeedSequence([2207, 12848, 55]))
    dirs = np.array([[1, 1, 1], [-1, 1, 1], [1, -1, -1]], np.float64) / np.sqrt(3.0)
    em = np.zeros(C)
    em[rng.choice(C, 4, replace=False)] = rng.uniform(0.5, 2.0, 4)
    w = dict(meshes=[mesh], dirs=dirs, G=1, kappa=rng.uniform(0.5, 5.0, (C, 1)),
             emission=em[:, None], boundary="vacuum", n_pbc=1, albedo=0.0, n_scat=1)
    a = oracle.forward(w)
    b = oracle.forward(dict(w, scheme="aligned"))
    assert _rel(b["J"], a["J"]) < 1e-14
    la = oracle.build_dag(mesh, dirs)
    lb = oracle.build_dag(mesh, dirs, scheme="aligned")
    for x, y in zip(la, lb):
        assert np.array_equal(x, y)


def test_aligned_conserves_photons():
    for w in (_w(200, 24, seed=56, albedo=0.5, n_scat=4), _w(180, 8, seed=57, periodic=True, n_pbc=4)):
        for law in ("upwind", "exp"):
            t = oracle.forward(dict(w, law=law))["totals"][0]
            lhs = t[:, 0] + t[:, 3] + t[:, 5]
            rhs = t[:, 1] + t[:, 2] + t[:, 4]
            assert np.all(np.abs(lhs - rhs) <= 1e-12 * t[:, 0])


def test_aligned_adjoint_matches_dense_and_central_differences():
    w = _w(140, 8, seed=58)
    gJ, gA = oracle.absorbed_loss_grads(w)
    dk, de = oracle.adjoint(w, gJ, gA)
    rk, re = DR.dense_adjoint(w, gJ, gA)
    assert _rel(dk, rk) < 1e-10 and _rel(de, re) < 1e-10
    kap0 = np.asarray(w["kappa"], np.float64).reshape(-1)
    h = 1e-6

    def loss(k):
        return oracle.forward(dict(w, kappa=k.reshape(-1, 1)))["absorbed"].sum() / (4 * np.pi)

    for c in (3, 50, 99):
        kp, km = kap0.copy(), kap0.copy()
        kp[c] *= 1 + h
        km[c] *= 1 - h
        fd = (loss(kp) - loss(km)) / (2 * h * kap0[c])
        assert abs(dk[c, 0] - fd) <= 1e-6 * abs(fd) + 1e-12


def test_aligned_periodic_adjoint_central_differences():
    w = _w(120, 8, seed=59, periodic=True, n_pbc=3, albedo=0.3, n_scat=2)
    gJ, gA = oracle.absorbed_loss_grads(w)
    dk, de = oracle.adjoint(w, gJ, gA)
    kap0 = np.asarray(w["kappa"], np.float64).reshape(-1)
    em0 = np.asarray(w["emission"], np.float64).reshape(-1)
    h = 1e-6

    def loss(k, e):
        return oracle.forward(dict(w, kappa=k.reshape(-1, 1), emission=e.reshape(-1, 1)))[
            "absorbed"].sum() / (4 * np.pi)

    for c in (7, 60):
        kp, km = kap0.copy(), kap0.copy()
        kp[c] *= 1 + h
        km[c] *= 1 - h
        fd = (loss(kp, em0) - loss(km, em0)) / (2 * h * kap0[c])
        assert abs(dk[c, 0] - fd) <= 1e-6 * abs(fd) + 1e-12
    for c in np.nonzero(em0)[0][:2]:
        ep, emm = em0.copy(), em0.copy()
        ep[c] *= 1 + h
        emm[c] *= 1 - h
        fd = (loss(kap0, ep) - loss(kap0, emm)) / (2 * h * em0[c])
        assert abs(de[c, 0] - fd) <= 1e-6 * abs(fd) + 1e-12


def test_aligned_needs_twins():
    w = _w(60, 4, seed=60)
    m = dict(w["meshes"][0])
    m.pop("face_twin")
    with pytest.raises(oracle.OracleError):
        oracle.forward(dict(w, meshes=[m]))

