"""Pins of the FP64 oracle against things other than itself: dense direct solves,
closed forms on lattices, conservation, acyclicity, finite differences."""
import numpy as np
import pytest

import oracle
from synth import workloads as W
from synth.directions import direction_set, octant_diagonals
from tests import dense_reference as DR


def _rel(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


@pytest.fixture(scope="module")
def tiny():
    return W.small_random(150, 8, G=2, seed=1, n_src=4)


# ----------------------------------------------------------------------------- dense solves
def test_forward_matches_dense_solve(tiny):
    r = oracle.forward(tiny, want_phi=True)
    ref = DR.dense_forward(tiny)
    assert _rel(r["phi"][0], ref["phi"][0]) < 1e-12
    assert _rel(r["J"], ref["J"]) < 1e-12
    assert _rel(r["absorbed"], ref["absorbed"]) < 1e-12
    assert _rel(r["totals"][..., :3], ref["totals"]) < 1e-12


def test_forward_dense_fibonacci_multimesh():
    w = W.small_random(120, 24, G=1, seed=2, n_meshes=3, n_src=2)
    r = oracle.forward(w, want_phi=True)
    ref = DR.dense_forward(w)
    for a, b in zip(r["phi"], ref["phi"]):
        assert _rel(a, b) < 1e-12
    assert _rel(r["J"], ref["J"]) < 1e-12


def test_forward_dense_many_faces():
    # every cell borders every other: long rows, cells with 105 faces
    w = W.many_faces(100, 24, G=2, seed=3)
    r = oracle.forward(w, want_phi=True)
    ref = DR.dense_forward(w)
    assert _rel(r["phi"][0], ref["phi"][0]) < 1e-12
    assert _rel(r["J"], ref["J"]) < 1e-12
    lv, order, indeg, depth = oracle.build_dag(w["meshes"][0], w["dirs"])
    for d in (0, 7, 23):
        assert np.array_equal(lv[d], DR.brute_levels(w["meshes"][0], w["dirs"][d])[0])


def test_periodic_passes_converge_to_cyclic_dense_solve():
    w = W.small_random(180, 8, G=1, seed=3, periodic=True, n_src=3, tau=2.0)
    ref = DR.dense_forward(w, cyclic=True)
    prev = None
    for n in (1, 2, 4, 8):
        w["n_pbc"] = n
        r = oracle.forward(w)
        if prev is not None:  # passes from a cold start increase monotonically
            assert np.all(r["J"] >= prev - 1e-15 * np.abs(prev))
        prev = r["J"]
    w["n_pbc"] = 200
    r = oracle.forward(w)
    assert _rel(r["J"], ref["J"]) < 1e-10
    t = r["totals"][0, 0]
    # converged: what leaves through the periodic faces comes back in
    assert abs(t[3] - t[4]) / t[4] < 1e-10
    assert t[6] < 1e-10


def test_periodic_uniform_medium_is_exact():
    """Uniform emissivity j and kappa in a fully periodic box: I = j/kappa everywhere."""
    w = W.small_random(150, 8, G=1, seed=4, periodic=True)
    mesh = w["meshes"][0]
    kap, jdens = 3.0, 2.0
    w["kappa"] = np.full((150, 1), kap)
    w["emission"] = (jdens * mesh["cell_volume"])[:, None]
    ref = DR.dense_forward(w, cyclic=True)
    D = len(w["dirs"])
    assert np.allclose(ref["phi"][0], jdens / (kap * D), rtol=1e-12)
    w["n_pbc"] = 400
    r = oracle.forward(w, want_phi=True)
    assert np.allclose(r["phi"][0], jdens / (kap * D), rtol=1e-9)


def test_scattering_iteration_converges_to_dense_system():
    w = W.small_random(100, 8, G=1, seed=5, n_src=2, albedo=0.5, n_scat=1)
    phi_fix = DR.dense_scatter_system(w)
    prev = None
    for n in (1, 2, 3, 5, 8, 60):
        w["n_scat"] = n
        r = oracle.forward(w, want_phi=True)
        if prev is not None:
            assert np.all(r["J"] >= prev * (1 - 1e-14))  # monotone from J = 0
        prev = r["J"]
    assert _rel(r["phi"][0][:, :, 0], phi_fix) < 1e-10
    # error contracts by at most the albedo per iteration
    w["n_scat"] = 4
    e4 = np.abs(oracle.forward(w)["J"][:, 0] - phi_fix.sum(0) / (4 * np.pi)).max()
    w["n_scat"] = 5
    e5 = np.abs(oracle.forward(w)["J"][:, 0] - phi_fix.sum(0) / (4 * np.pi)).max()
    assert e5 <= 0.5 * e4 * (1 + 1e-9)


# ----------------------------------------------------------------------------- closed forms
def test_lattice_levels_closed_form():
    n = 6
    dirs = octant_diagonals()
    w = W.lattice_workload(n, dirs, 1.0, [0], [1.0])
    lv, order, indeg, depth = oracle.build_dag(w["meshes"][0], dirs)
    cid = np.arange(n ** 3)
    i, j, k = cid % n, (cid // n) % n, cid // (n * n)
    for d, om in enumerate(dirs):
        ii = np.where(om[0] > 0, i, n - 1 - i)
        jj = np.where(om[1] > 0, j, n - 1 - j)
        kk = np.where(om[2] > 0, k, n - 1 - k)
        assert np.array_equal(lv[d], ii + jj + kk)
        assert depth[d] == 3 * n - 2
        assert np.array_equal(indeg[d], (ii > 0).astype(int) + (jj > 0) + (kk > 0))
    # axis-aligned: level = i, transverse faces carry nothing
    lv, _, indeg, depth = oracle.build_dag(w["meshes"][0], np.array([[1.0, 0.0, 0.0]]))
    assert np.array_equal(lv[0], i) and depth[0] == n
    assert np.array_equal(indeg[0], (i > 0).astype(int))


@pytest.mark.parametrize("kappa", [0.5, 3.0])
def test_aligned_beam_closed_form(kappa):
    """Omega = +x on a lattice: phi_m = phi_0 (1 + kappa h)^-m, phi_0 = (L/D)/(h^2 + kappa h^3)."""
    n = 8
    h = 1.0 / n
    src = [0 + n * (3 + n * 5)]  # cell (0,3,5)
    w = W.lattice_workload(n, np.array([[1.0, 0.0, 0.0]]), kappa, src, [2.0])
    r = oracle.forward(w, want_phi=True)
    phi = r["phi"][0][0, :, 0]
    row = [m + n * (3 + n * 5) for m in range(n)]
    kappa = float(w["kappa"][0, 0])  # inputs are rounded to FP32 once
    phi0 = 2.0 / (h * h + kappa * h ** 3)
    expect = phi0 * (1.0 + kappa * h) ** -np.arange(n)
    assert _rel(phi[row], expect) < 1e-13
    mask = np.ones(n ** 3, bool)
    mask[row] = False
    assert np.all(phi[mask] == 0.0)
    t = r["totals"][0, 0]
    assert abs(t[2] - h * h * phi[row[-1]]) < 1e-13 * t[0]


def test_beam_converges_to_exponential_attenuation():
    """Transmission through a slab of optical depth kappa*L converges to exp(-kappa L) at first order."""
    kappa = 2.0
    errs = []
    for n in (4, 8, 16):
        h = 1.0 / n
        w = W.lattice_workload(n, np.array([[1.0, 0.0, 0.0]]), kappa, [0], [1.0])
        r = oracle.forward(w, want_phi=True)
        phi = r["phi"][0][0, :, 0]
        trans = phi[n - 1] / phi[0]  # attenuation over (n-1) cells of width h
        errs.append(abs(trans - np.exp(-kappa * (n - 1) * h)))
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]


def test_single_cell_closed_form():
    dirs = direction_set(24)
    w = W.lattice_workload(1, dirs, 0.7, [0], [3.0])
    r = oracle.forward(w, want_phi=True)
    aperp = np.abs(dirs).sum(axis=1)
    kap = float(w["kappa"][0, 0])  # inputs are rounded to FP32 once
    expect = (3.0 / 24) / (aperp + kap)
    assert _rel(r["phi"][0][:, 0, 0], expect) < 1e-14


# ----------------------------------------------------------------------------- conservation
def test_conservation_and_limits():
    w = W.small_random(600, 24, G=3, seed=6, n_src=5, n_meshes=2)
    r = oracle.forward(w)
    t = r["totals"]
    assert np.all(np.abs(t[..., 0] - t[..., 1] - t[..., 2]) <= 1e-13 * t[..., 0])
    assert np.all(r["J"] >= 0)
    w0 = dict(w, kappa=np.zeros_like(w["kappa"]))
    t0 = oracle.forward(w0)["totals"]
    assert np.all(t0[..., 1] == 0) and np.allclose(t0[..., 2], t0[..., 0], rtol=1e-13)
    wbig = dict(w, kappa=np.full_like(w["kappa"], 1e9))
    rb = oracle.forward(wbig)
    em = np.asarray(w["emission"], np.float64)
    # leakage out of a cell is ~ Aperp/(kappa V) ~ 1e-7 of its source at kappa = 1e9
    assert np.allclose(rb["absorbed"], em, rtol=1e-5, atol=1e-5 * em.max())


def test_conservation_with_scattering_and_periodic_passes():
    w = W.small_random(400, 8, G=2, seed=7, periodic=True, n_src=3, albedo=0.5, n_scat=4, n_pbc=3)
    t = oracle.forward(w)["totals"][0]
    lhs = t[:, 0] + t[:, 3] + t[:, 5]
    rhs = t[:, 1] + t[:, 2] + t[:, 4]
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * t[:, 0])
    assert np.all(t[:, 2] == 0)  # no walls in a periodic box


# ----------------------------------------------------------------------------- DAG
def test_dag_matches_brute_force_levels():
    w = W.small_random(500, 24, seed=8)
    mesh = w["meshes"][0]
    lv, order, indeg, depth = oracle.build_dag(mesh, w["dirs"])
    for d in range(0, 24, 5):
        ref, src, dst = DR.brute_levels(mesh, w["dirs"][d])
        assert np.array_equal(lv[d], ref)
        assert np.array_equal(indeg[d], np.bincount(dst, minlength=500))
        assert depth[d] == ref.max() + 1
        # canonical order: sorted by (level, cell)
        assert np.array_equal(order[d], np.lexsort((np.arange(500), ref)))


def test_reversed_direction_is_transpose_and_acyclic():
    w = W.small_random(800, 48, seed=9)
    mesh = w["meshes"][0]
    dirs = w["dirs"]
    both = np.concatenate([dirs, -dirs])
    lv, order, indeg, depth = oracle.build_dag(mesh, both)  # raises on any cycle (appendix A)
    fp = mesh["face_ptr"]
    owner = np.repeat(np.arange(800), np.diff(fp))
    for d in range(0, 48, 7):
        s = mesh["face_normal"] @ dirs[d]
        outdeg = np.bincount(owner[(s > 1e-12) & (mesh["face_nbr"] >= 0)], minlength=800)
        assert np.array_equal(indeg[48 + d], outdeg)
        assert indeg[d].sum() == np.count_nonzero((s < -1e-12) & (mesh["face_nbr"] >= 0))


def test_cyclic_graph_is_reported():
    w = W.small_random(200, 8, seed=10, periodic=True)
    mesh = dict(w["meshes"][0], periodic=False)  # keep wrap-around faces in the graph
    with pytest.raises(oracle.OracleError, match="cyclic"):
        oracle.build_dag(mesh, w["dirs"])
    with pytest.raises(oracle.OracleError, match="cyclic"):
        oracle.forward(dict(w, meshes=[mesh], boundary="vacuum"))


# ----------------------------------------------------------------------------- adjoint
def _loss(w):
    r = oracle.forward(w)
    return r["absorbed"].sum() / (4 * np.pi)


def test_adjoint_matches_dense_adjoint():
    w = W.small_random(150, 8, G=2, seed=11, n_src=4)
    rng = np.random.default_rng(0)
    gJ = rng.random((150, 2))
    gA = rng.random((150, 2))
    dk, de = oracle.adjoint(w, gJ, gA)
    rk, re_ = DR.dense_adjoint(w, gJ, gA)
    assert _rel(dk, rk) < 1e-11
    assert _rel(de, re_) < 1e-11


@pytest.mark.parametrize("albedo,n_scat", [(0.0, 1), (0.5, 5)])
def test_adjoint_central_differences(albedo, n_scat):
    w = W.small_random(200, 8, G=1, seed=12, n_src=3, albedo=albedo, n_scat=n_scat)
    w["kappa"] = np.asarray(w["kappa"], np.float64)
    w["emission"] = np.asarray(w["emission"], np.float64)
    gJ, gA = oracle.absorbed_loss_grads(w)
    dk, de = oracle.adjoint(w, gJ, gA)
    rng = np.random.default_rng(1)
    h = 1e-6
    cells = rng.choice(200, 8, replace=False)
    for c in cells:
        k0 = w["kappa"][c, 0]
        wp = dict(w, kappa=w["kappa"].copy())
        wm = dict(w, kappa=w["kappa"].copy())
        wp["kappa"][c, 0] = k0 * (1 + h)
        wm["kappa"][c, 0] = k0 * (1 - h)
        fd = (_loss(wp) - _loss(wm)) / (2 * h * k0)
        assert abs(fd - dk[c, 0]) <= 1e-6 * abs(dk[c, 0]) + 1e-10 * _loss(w) / k0
    for c in w["sources"]:
        L0 = w["emission"][c, 0]
        wp = dict(w, emission=w["emission"].copy())
        wm = dict(w, emission=w["emission"].copy())
        wp["emission"][c, 0] = L0 * (1 + h)
        wm["emission"][c, 0] = L0 * (1 - h)
        fd = (_loss(wp) - _loss(wm)) / (2 * h * L0)
        assert abs(fd - de[c, 0]) <= 1e-6 * abs(de[c, 0])
    # every source photon is absorbed or escapes: 0 <= dL/dL_c <= 1/(4 pi)
    assert np.all(de >= 0) and np.all(de <= 1 / (4 * np.pi) * (1 + 1e-12))


def test_adjoint_sign_for_mean_intensity_loss():
    """For L = sum J, raising kappa anywhere can only lower J (M-matrix): dL/dkappa <= 0."""
    w = W.small_random(200, 24, G=1, seed=13, n_src=3)
    dk, _ = oracle.adjoint(w, np.ones((200, 1)), np.zeros((200, 1)))
    assert np.all(dk <= 0)


@pytest.mark.parametrize("law,albedo,n_scat", [("upwind", 0.0, 1), ("upwind", 0.4, 3), ("exp", 0.4, 2)])
def test_periodic_adjoint_central_differences(law, albedo, n_scat):
    """Adjoint through 3 periodic passes (and source iterations): central differences."""
    w = W.small_random(200, 8, G=1, seed=14, periodic=True, n_pbc=3, n_src=3, albedo=albedo,
                       n_scat=n_scat, tau=2.0)
    w = dict(w, law=law, kappa=np.asarray(w["kappa"], np.float64),
             emission=np.asarray(w["emission"], np.float64))
    gJ, gA = oracle.absorbed_loss_grads(w)
    dk, de = oracle.adjoint(w, gJ, gA)
    L = _loss(w)
    rng = np.random.default_rng(4)
    h = 1e-6
    for c in rng.choice(200, 8, replace=False):
        k0 = w["kappa"][c, 0]
        wp = dict(w, kappa=w["kappa"].copy())
        wm = dict(w, kappa=w["kappa"].copy())
        wp["kappa"][c, 0] = k0 * (1 + h)
        wm["kappa"][c, 0] = k0 * (1 - h)
        fd = (_loss(wp) - _loss(wm)) / (2 * h * k0)
        assert abs(fd - dk[c, 0]) <= 1e-6 * abs(dk[c, 0]) + 1e-10 * L / k0
    for c in w["sources"]:
        L0 = w["emission"][c, 0]
        wp = dict(w, emission=w["emission"].copy())
        wm = dict(w, emission=w["emission"].copy())
        wp["emission"][c, 0] = L0 * (1 + h)
        wm["emission"][c, 0] = L0 * (1 - h)
        fd = (_loss(wp) - _loss(wm)) / (2 * h * L0)
        assert abs(fd - de[c, 0]) <= 1e-6 * abs(de[c, 0])


@pytest.mark.parametrize("law,n_pbc,n_scat", [("upwind", 3, 3), ("upwind", 2, 4), ("exp", 4, 2)])
def test_merged_adjoint_central_differences(law, n_pbc, n_scat):
    """Adjoint of the merged order (each pass takes its scattering source and its
    periodic inflow from the pass before): central differences of the merged
    forward, and different from the nested order's gradients."""
    w = W.small_random(200, 8, G=1, seed=15, periodic=True, n_pbc=n_pbc, n_src=3, albedo=0.4,
                       n_scat=n_scat, tau=2.0)
    w = dict(w, law=law, merge=True, kappa=np.asarray(w["kappa"], np.float64),
             emission=np.asarray(w["emission"], np.float64))
    gJ, gA = oracle.absorbed_loss_grads(w)
    dk, de = oracle.adjoint(w, gJ, gA)
    dkn, _ = oracle.adjoint(dict(w, merge=False), gJ, gA)
    assert _rel(dk, dkn) > 1e-6  # the orders differ, and so do their gradients
    L = _loss(w)
    rng = np.random.default_rng(5)
    h = 1e-6
    for c in rng.choice(200, 8, replace=False):
        k0 = w["kappa"][c, 0]
        wp = dict(w, kappa=w["kappa"].copy())
        wm = dict(w, kappa=w["kappa"].copy())
        wp["kappa"][c, 0] = k0 * (1 + h)
        wm["kappa"][c, 0] = k0 * (1 - h)
        fd = (_loss(wp) - _loss(wm)) / (2 * h * k0)
        assert abs(fd - dk[c, 0]) <= 1e-6 * abs(dk[c, 0]) + 1e-10 * L / k0
    for c in w["sources"]:
        L0 = w["emission"][c, 0]
        wp = dict(w, emission=w["emission"].copy())
        wm = dict(w, emission=w["emission"].copy())
        wp["emission"][c, 0] = L0 * (1 + h)
        wm["emission"][c, 0] = L0 * (1 - h)
        fd = (_loss(wp) - _loss(wm)) / (2 * h * L0)
        assert abs(fd - de[c, 0]) <= 1e-6 * abs(de[c, 0])


@pytest.mark.parametrize("merge,n_pbc,n_scat", [(False, 3, 1), (False, 2, 3), (True, 2, 3)])
def test_warm_start_adjoint_central_differences(merge, n_pbc, n_scat):
    """Warm start (the first pass's periodic inflow taken from an earlier run's
    exit values, held fixed): adjoint against central differences of the forward
    with the same inflow, and different from the adjoint from zero inflow."""
    w = W.small_random(200, 8, G=1, seed=16, periodic=True, n_pbc=n_pbc, n_src=3, albedo=0.4,
                       n_scat=n_scat, tau=2.0)
    w = dict(w, merge=merge, kappa=np.asarray(w["kappa"], np.float64),
             emission=np.asarray(w["emission"], np.float64))
    warm = oracle.forward(dict(w, kappa=w["kappa"] * 1.3), want_phi=True)["phi"]
    gJ, gA = oracle.absorbed_loss_grads(w)
    dk, de = oracle.adjoint(w, gJ, gA, phi_init=warm)
    dk0, _ = oracle.adjoint(w, gJ, gA)
    assert _rel(dk, dk0) > 1e-6

    def loss(ww):
        return oracle.forward(ww, phi_init=warm)["absorbed"].sum() / (4 * np.pi)

    L = loss(w)
    rng = np.random.default_rng(7)
    h = 1e-6
    for c in rng.choice(200, 8, replace=False):
        k0 = w["kappa"][c, 0]
        wp = dict(w, kappa=w["kappa"].copy())
        wm = dict(w, kappa=w["kappa"].copy())
        wp["kappa"][c, 0] = k0 * (1 + h)
        wm["kappa"][c, 0] = k0 * (1 - h)
        fd = (loss(wp) - loss(wm)) / (2 * h * k0)
        assert abs(fd - dk[c, 0]) <= 1e-6 * abs(dk[c, 0]) + 1e-10 * L / k0
    for c in w["sources"]:
        L0 = w["emission"][c, 0]
        wp = dict(w, emission=w["emission"].copy())
        wm = dict(w, emission=w["emission"].copy())
        wp["emission"][c, 0] = L0 * (1 + h)
        wm["emission"][c, 0] = L0 * (1 - h)
        fd = (loss(wp) - loss(wm)) / (2 * h * L0)
        assert abs(fd - de[c, 0]) <= 1e-6 * abs(de[c, 0])


@pytest.mark.parametrize("tol,n_scat,same_as", [(0.25, 2, 6), (0.3, 3, None)])
def test_pbc_tol_adjoint_central_differences(tol, n_scat, same_as):
    """With pbc_tol the forward ends each iteration's passes once E < pbc_tol; the
    adjoint runs the passes the forward ran (the counts held fixed): central
    differences of the same forward, and with one count in every iteration the
    adjoint of that fixed count, exactly."""
    w = W.small_random(200, 8, G=1, seed=17, periodic=True, n_pbc=10, n_src=3, albedo=0.4,
                       n_scat=n_scat, tau=2.0)
    w = dict(w, pbc_tol=tol, kappa=np.asarray(w["kappa"], np.float64),
             emission=np.asarray(w["emission"], np.float64))
    gJ, gA = oracle.absorbed_loss_grads(w)
    dk, de = oracle.adjoint(w, gJ, gA)
    if same_as is not None:
        dkf, def_ = oracle.adjoint(dict(w, pbc_tol=0.0, n_pbc=same_as), gJ, gA)
        assert np.array_equal(dk, dkf) and np.array_equal(de, def_)
    L = _loss(w)
    rng = np.random.default_rng(8)
    # ten passes carry more rounding into the loss than the three of the other
    # pins: a step of 1e-5 keeps it below the bound (the O(h^2) truncation stays
    # near 1e-10 relative, and no stopping decision moves)
    h = 1e-5
    for c in rng.choice(200, 8, replace=False):
        k0 = w["kappa"][c, 0]
        wp = dict(w, kappa=w["kappa"].copy())
        wm = dict(w, kappa=w["kappa"].copy())
        wp["kappa"][c, 0] = k0 * (1 + h)
        wm["kappa"][c, 0] = k0 * (1 - h)
        fd = (_loss(wp) - _loss(wm)) / (2 * h * k0)
        assert abs(fd - dk[c, 0]) <= 1e-6 * abs(dk[c, 0]) + 1e-10 * L / k0
    for c in w["sources"]:
        L0 = w["emission"][c, 0]
        wp = dict(w, emission=w["emission"].copy())
        wm = dict(w, emission=w["emission"].copy())
        wp["emission"][c, 0] = L0 * (1 + h)
        wm["emission"][c, 0] = L0 * (1 - h)
        fd = (_loss(wp) - _loss(wm)) / (2 * h * L0)
        assert abs(fd - de[c, 0]) <= 1e-6 * abs(de[c, 0])


def test_periodic_adjoint_converges_to_the_cyclic_adjoint():
    """Many passes: the gradients of the passes approach those of the cyclic fixed point."""
    w = W.small_random(180, 8, G=1, seed=3, periodic=True, n_src=3, tau=2.0)
    rng = np.random.default_rng(6)
    gJ = rng.random((180, 1))
    gA = rng.random((180, 1))
    rk, re_ = DR.dense_adjoint(w, gJ, gA, cyclic=True)
    dk, de = oracle.adjoint(dict(w, n_pbc=200), gJ, gA)
    assert _rel(dk, rk) < 1e-9
    assert _rel(de, re_) < 1e-9
