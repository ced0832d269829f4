"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on identical seeded inputs.

Tolerances: dependency graphs (levels, canonical order, upwind counts) bit-exact;
J and absorbed within 1e-5 relative elementwise wherever the FP64 value is at least
1e-20 of its maximum (FP32 headroom) and within 1e-5 in relative L1; FP64 totals
within 1e-5 relative; GPU photon balance within 1e-6 relative; gradients within
1e-5 in relative L2 and elementwise within 1e-4 relative plus 1e-6 of the largest
magnitude (dL/dkappa is a difference of two terms carried in FP32).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from synth import workloads as W  # noqa: E402
from synth.directions import direction_set  # noqa: E402

REL = 1e-5


def _sw():
    import paper_2207_12848_amd as sw
    return sw


def _dev(w):
    G = w["G"]
    k = torch.tensor(np.asarray(w["kappa"], np.float32).reshape(-1, G), device="cuda")
    e = torch.tensor(np.asarray(w["emission"], np.float32).reshape(-1, G), device="cuda")
    return k, e


def _opts(w):
    return dict(boundary=w["boundary"], n_pbc=w["n_pbc"], albedo=w["albedo"], n_scat=w["n_scat"],
                law=w.get("law", "upwind"))


def assert_field_close(gpu, ref, rel=REL, floor=1e-20, name="field"):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert gpu.shape == ref.shape
    assert np.all(np.isfinite(gpu))
    big = np.abs(ref) >= floor * np.abs(ref).max()
    err = np.abs(gpu - ref)
    worst = (err[big] / np.abs(ref[big])).max() if big.any() else 0.0
    assert worst <= rel, "%s: max rel err %.3e" % (name, worst)
    l1 = err.sum() / max(np.abs(ref).sum(), 1e-300)
    assert l1 <= rel, "%s: rel L1 err %.3e" % (name, l1)


def run_gpu(w, form="batched", **kw):
    sw = _sw()
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    J, A, tot = sw.forward(dag, k, e, form=form, **_opts(w), **kw)
    torch.cuda.synchronize()
    return dag, J.cpu().numpy(), A.cpu().numpy(), tot.cpu().numpy()


def check_forward(w, **kw):
    dag, J, A, tot = run_gpu(w, **kw)
    ref = oracle.forward(w)
    assert_field_close(J, ref["J"], name="J")
    assert_field_close(A, ref["absorbed"], name="absorbed")
    t, rt = tot, ref["totals"]
    for k in (0, 1, 2, 3, 4):
        scale = np.maximum(np.abs(rt[..., k]), 1e-12 * rt[..., 0])
        assert np.all(np.abs(t[..., k] - rt[..., k]) <= REL * scale + 1e-300), k
    # photon balance of the GPU's own FP64 totals
    lhs = t[..., 0] + t[..., 3] + t[..., 5]
    rhs = t[..., 1] + t[..., 2] + t[..., 4]
    assert np.all(np.abs(lhs - rhs) <= 1e-6 * t[..., 0])
    return dag, J, A, tot, ref


# ----------------------------------------------------------------------------- DAG
@pytest.mark.parametrize("case", ["c1", "multi", "periodic"])
def test_dag_bit_exact(case):
    sw = _sw()
    if case == "c1":
        w = W.c1_plain_small()
    elif case == "multi":
        w = W.small_random(700, 24, seed=21, n_meshes=4)
    else:
        w = W.small_random(900, 48, seed=22, periodic=True)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    lv, od, ind = dag.export()
    for m, mesh in enumerate(w["meshes"]):
        rl, ro, ri, rd = oracle.build_dag(mesh, w["dirs"])
        assert np.array_equal(dag.split(lv)[m], rl)
        assert np.array_equal(dag.split(od)[m], ro)
        assert np.array_equal(dag.split(ind)[m], ri)
    info = dag.info()
    assert info["n_tasks"] == sum(len(m["cell_volume"]) for m in w["meshes"]) * len(w["dirs"])


def test_cycle_is_reported():
    sw = _sw()
    w = W.small_random(300, 8, seed=23, periodic=True)
    mesh = dict(w["meshes"][0], periodic=False)  # wrap-around faces kept in the graph
    with pytest.raises(sw.SweepError, match="CYCLE"):
        sw.build_dag([mesh], w["dirs"])


def test_invalid_mesh_is_rejected():
    sw = _sw()
    w = W.small_random(200, 8, seed=24)
    mesh = dict(w["meshes"][0])
    mesh["face_normal"] = mesh["face_normal"] * 1.01
    with pytest.raises(sw.SweepError, match="INVALID_ARG"):
        sw.build_dag([mesh], w["dirs"])
    with pytest.raises(sw.SweepError, match="INVALID_ARG"):
        sw.build_dag(w["meshes"], w["dirs"] * 1.1)


# ----------------------------------------------------------------------------- forward
def test_forward_c1():
    check_forward(W.c1_plain_small())


@pytest.mark.parametrize("G", [1, 2, 4, 6])
def test_forward_groups_multimesh(G):
    w = W.small_random(1500, 24, G=G, seed=30 + G, n_meshes=3, n_src=5)
    check_forward(w)


def test_forward_plain_equals_batched_bitwise():
    # the plain form (one group per launch) and the batched form (groups packed
    # per task) perform the same FP32 operations in the same order
    w = W.small_random(2000, 24, G=3, seed=40, n_meshes=2)
    _, J1, A1, _ = run_gpu(w, form="batched")
    _, J2, A2, _ = run_gpu(w, form="plain")
    assert np.array_equal(J1, J2) and np.array_equal(A1, A2)
    # a small ring adds the inflow of ring misses after the rest of the row: the
    # same terms in another order, so equal to FP32 rounding of the sums
    _, J3, A3, _ = run_gpu(w, form="batched", block=256, ring=256)
    for x, y in ((J3, J1), (A3, A1)):
        big = np.abs(y) >= 1e-20 * np.abs(y).max()
        assert (np.abs(x - y)[big] / np.abs(y)[big]).max() <= 2e-6


def test_forward_deterministic():
    w = W.small_random(3000, 48, G=1, seed=41)
    _, J1, A1, t1 = run_gpu(w)
    _, J2, A2, t2 = run_gpu(w)
    assert np.array_equal(J1, J2) and np.array_equal(A1, A2) and np.array_equal(t1, t2)


def test_forward_small_ring_uses_global_fallback():
    w = W.small_random(4000, 8, G=2, seed=42)
    check_forward(w, ring=64, block=256)


def test_forward_periodic_passes():
    w = W.small_random(3000, 24, G=2, seed=43, periodic=True, n_pbc=3, n_src=6)
    dag, J, A, tot, ref = check_forward(w)
    rt = ref["totals"]
    assert np.allclose(tot[..., 6], rt[..., 6], rtol=1e-4, atol=1e-6)
    assert np.allclose(tot[..., 7], rt[..., 7], rtol=1e-4, atol=1e-8)


def test_forward_scattering_iterations():
    w = W.small_random(2500, 24, G=1, seed=44, n_src=4, albedo=0.5, n_scat=6, n_meshes=2)
    dag, J, A, tot, ref = check_forward(w)
    assert np.allclose(tot[..., 5], ref["totals"][..., 5], rtol=1e-4)


def test_forward_periodic_and_scattering():
    w = W.small_random(2000, 8, G=2, seed=45, periodic=True, n_pbc=2, albedo=0.3, n_scat=3)
    check_forward(w)


def test_forward_edge_cases():
    # single cell, no faces between cells
    w = W.lattice_workload(1, direction_set(24), 0.5, [0], [1.0])
    check_forward(w)
    # zero emission everywhere: all outputs exactly zero
    w = W.small_random(500, 8, seed=46)
    w["emission"] = np.zeros_like(w["emission"])
    _, J, A, tot = run_gpu(w)
    assert not J.any() and not A.any() and not tot[..., :6].any()
    # kappa = 0: nothing absorbed
    w = W.small_random(500, 8, seed=47)
    w["kappa"] = np.zeros_like(w["kappa"])
    _, J, A, tot = run_gpu(w)
    assert not A.any()
    assert abs(tot[0, 0, 2] - tot[0, 0, 0]) <= 1e-6 * tot[0, 0, 0]


def test_many_faces_rows_and_tiles():
    # cells with 105 faces: face tiles read from global memory, downwind rows
    # continued in overflow lists, face classes past the 32 face bits, upwind
    # counts past the 4-bit LDS counters
    sw = _sw()
    w = W.many_faces(100, 24, G=2, seed=4, albedo=0.3, n_scat=2)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    lv, od, ind = dag.export()
    level, order, indeg, depth = oracle.build_dag(w["meshes"][0], w["dirs"])
    assert np.array_equal(lv, level.reshape(-1))
    assert np.array_equal(od, order.reshape(-1))
    assert np.array_equal(ind, indeg.reshape(-1))
    assert indeg.max() > 32  # the graph really has long rows
    check_forward(w)
    C = 100
    rng = np.random.default_rng(6)
    gJ = rng.random((C, 2)).astype(np.float32)
    gA = rng.random((C, 2)).astype(np.float32)
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA)
    k, e = _dev(w)
    J, A, tot, saved = sw.forward(dag, k, e, save_for_adjoint=True, **_opts(w))
    dk, de = sw.adjoint(dag, k, e, saved, torch.tensor(gJ, device="cuda"),
                        torch.tensor(gA, device="cuda"), **_opts(w))
    _grad_close(dk.cpu().numpy(), dk_ref)
    _grad_close(de.cpu().numpy(), de_ref)


def test_forward_lattice_beam():
    n = 12
    w = W.lattice_workload(n, np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0]]), 1.5,
                           [n // 2 + n * (n // 2 + n * (n // 2))], [1.0])
    check_forward(w)


# ----------------------------------------------------------------------------- adjoint
def _grad_close(g, r):
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    l2 = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)
    assert l2 <= 1e-5, "rel L2 %.3e" % l2
    # relative where the gradient is large, absolute (1e-6 of the largest) where
    # it is a small difference of the absorption and transport terms
    excess = np.abs(g - r) - (1e-4 * np.abs(r) + 1e-6 * np.abs(r).max())
    assert excess.max() <= 0.0, "elementwise excess %.3e" % excess.max()


@pytest.mark.parametrize("albedo,n_scat,G", [(0.0, 1, 1), (0.0, 1, 3), (0.5, 4, 1)])
def test_adjoint_matches_oracle(albedo, n_scat, G):
    sw = _sw()
    w = W.small_random(2000, 24, G=G, seed=50 + n_scat, n_src=4, albedo=albedo, n_scat=n_scat,
                       n_meshes=2)
    rng = np.random.default_rng(5)
    C = sum(len(m["cell_volume"]) for m in w["meshes"])
    gJ = rng.random((C, G)).astype(np.float32)
    gA = rng.random((C, G)).astype(np.float32)
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    J, A, tot, saved = sw.forward(dag, k, e, save_for_adjoint=True, **_opts(w))
    dk, de = sw.adjoint(dag, k, e, saved, torch.tensor(gJ, device="cuda"),
                        torch.tensor(gA, device="cuda"), **_opts(w))
    _grad_close(dk.cpu().numpy(), dk_ref)
    _grad_close(de.cpu().numpy(), de_ref)


def test_autograd_function():
    sw = _sw()
    w = W.small_random(1500, 24, G=1, seed=60, n_src=3)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    k.requires_grad_(True)
    e.requires_grad_(True)
    J, A, tot = sw.SweepFunction.apply(k, e, dag, _opts(w))
    loss = A.sum() / (4 * np.pi)
    loss.backward()
    gJ, gA = oracle.absorbed_loss_grads(w)
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA)
    _grad_close(k.grad.cpu().numpy(), dk_ref)
    _grad_close(e.grad.cpu().numpy(), de_ref)


@pytest.mark.parametrize("law,n_pbc,albedo,n_scat,G", [("upwind", 3, 0.0, 1, 1), ("upwind", 2, 0.4, 3, 2),
                                                      ("exp", 3, 0.3, 2, 1)])
def test_periodic_adjoint_matches_oracle(law, n_pbc, albedo, n_scat, G):
    sw = _sw()
    w = W.small_random(2000, 24, G=G, seed=61 + n_pbc, periodic=True, n_pbc=n_pbc, n_src=4,
                       albedo=albedo, n_scat=n_scat, tau=2.0)
    w = dict(w, law=law)
    rng = np.random.default_rng(12)
    C = len(w["meshes"][0]["cell_volume"])
    gJ = rng.random((C, G)).astype(np.float32)
    gA = rng.random((C, G)).astype(np.float32)
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    J, A, tot, saved = sw.forward(dag, k, e, save_for_adjoint=True, **_opts(w))
    dk, de = sw.adjoint(dag, k, e, saved, torch.tensor(gJ, device="cuda"),
                        torch.tensor(gA, device="cuda"), **_opts(w))
    _grad_close(dk.cpu().numpy(), dk_ref)
    _grad_close(de.cpu().numpy(), de_ref)


def test_periodic_several_meshes_forward_and_adjoint():
    """Three periodic meshes of different sizes in one DAG: the periodic half-face
    lists, their per-direction weights and tasks are built mesh by mesh and the
    folds address partners by global cell id; forward (with E) and adjoint
    against the oracle."""
    sw = _sw()
    w = W.small_random(1500, 24, G=2, seed=64, periodic=True, n_pbc=3, n_meshes=3, n_src=4, tau=2.0)
    dag, J, A, tot, ref = check_forward(w)
    rt = ref["totals"]
    assert np.allclose(tot[..., 3], rt[..., 3], rtol=1e-5)
    assert np.allclose(tot[..., 6], rt[..., 6], rtol=1e-4, atol=1e-6)
    C = sum(len(m["cell_volume"]) for m in w["meshes"])
    rng = np.random.default_rng(13)
    gJ = rng.random((C, 2)).astype(np.float32)
    gA = rng.random((C, 2)).astype(np.float32)
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA)
    k, e = _dev(w)
    J, A, tot, saved = sw.forward(dag, k, e, save_for_adjoint=True, **_opts(w))
    dk, de = sw.adjoint(dag, k, e, saved, torch.tensor(gJ, device="cuda"),
                        torch.tensor(gA, device="cuda"), **_opts(w))
    _grad_close(dk.cpu().numpy(), dk_ref)
    _grad_close(de.cpu().numpy(), de_ref)


def test_periodic_adjoint_of_pbc_tol_is_not_captured():
    sw = _sw()
    w = W.small_random(800, 8, seed=61, periodic=True, n_pbc=3)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    # pbc_tol's pass counts come from the workspace: no graph capture
    J, A, tot, saved = sw.forward(dag, k, e, save_for_adjoint=True, boundary="periodic", n_pbc=3,
                                  pbc_tol=0.1)
    with pytest.raises(sw.SweepError, match="INVALID_ARG"):
        sw.adjoint(dag, k, e, saved, torch.ones_like(k), torch.ones_like(k),
                   boundary="periodic", n_pbc=3, pbc_tol=0.1, use_graph=True)
