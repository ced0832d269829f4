"""GPU parity of the merged periodic/scattering iterations and the warm-started
periodic inflow (sec. 2.7) against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from synth import workloads as W  # noqa: E402
from tests.test_gpu_parity import (_dev, _grad_close, _opts, _sw, assert_field_close,  # noqa: E402
                                   check_forward)


@pytest.mark.parametrize("law,n_pbc,n_scat", [("upwind", 3, 5), ("exp", 6, 2), ("upwind", 4, 4)])
def test_merged_iterations_match_oracle(law, n_pbc, n_scat):
    w = W.small_random(2500, 24, G=2, seed=90 + n_pbc, periodic=True, n_pbc=n_pbc, albedo=0.5,
                       n_scat=n_scat, n_src=5)
    w = dict(w, law=law, merge=True)
    dag, J, A, tot, ref = check_forward(w, merge=True)
    assert np.allclose(tot[..., 6], ref["totals"][..., 6], rtol=1e-4, atol=1e-6)
    assert np.allclose(tot[..., 5], ref["totals"][..., 5], rtol=1e-4, atol=1e-8 * tot[..., 0].max())


@pytest.mark.parametrize("law,n_pbc,n_scat,G", [("upwind", 3, 3, 2), ("upwind", 2, 4, 1), ("exp", 4, 2, 1)])
def test_merged_adjoint_matches_oracle(law, n_pbc, n_scat, G):
    """The adjoint of the merged order (every pass recomputed, then reversed with
    its own scattering source gradient and the later pass's lambda through the
    periodic faces) against the oracle's, with random loss gradients."""
    sw = _sw()
    w = W.small_random(2000, 24, G=G, seed=97 + n_pbc, periodic=True, n_pbc=n_pbc, albedo=0.4,
                       n_scat=n_scat, n_src=4, tau=2.0)
    w = dict(w, law=law, merge=True)
    rng = np.random.default_rng(14)
    C = len(w["meshes"][0]["cell_volume"])
    gJ = rng.random((C, G)).astype(np.float32)
    gA = rng.random((C, G)).astype(np.float32)
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    J, A, tot, saved = sw.forward(dag, k, e, save_for_adjoint=True, merge=True, **_opts(w))
    dk, de = sw.adjoint(dag, k, e, saved, torch.tensor(gJ, device="cuda"),
                        torch.tensor(gA, device="cuda"), merge=True, **_opts(w))
    _grad_close(dk.cpu().numpy(), dk_ref)
    _grad_close(de.cpu().numpy(), de_ref)
    # the merged gradients are not the nested order's
    dkn, _ = sw.adjoint(dag, k, e, sw.forward(dag, k, e, save_for_adjoint=True, **_opts(w))[3],
                        torch.tensor(gJ, device="cuda"), torch.tensor(gA, device="cuda"), **_opts(w))
    assert not torch.equal(dk, dkn)


def test_merged_equals_nested_without_scattering():
    sw = _sw()
    w = W.small_random(1500, 8, G=1, seed=95, periodic=True, n_pbc=4)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    a = sw.forward(dag, k, e, **_opts(w))
    b = sw.forward(dag, k, e, merge=True, **_opts(w))
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_warm_start_matches_oracle_and_continues_the_passes():
    sw = _sw()
    w = W.small_random(3000, 24, G=2, seed=96, periodic=True, n_src=6, tau=2.0)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    # one workspace for both calls, sized for the larger (it keeps every pass's phi)
    import ctypes
    nbytes = sw.sweep_saved_bytes(dag.handle, 2, ctypes.byref(sw._fwd_opts(boundary="periodic", n_pbc=4)))
    saved = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    sw.forward(dag, k, e, saved=saved, boundary="periodic", n_pbc=3)
    J, A, tot, _ = sw.forward(dag, k, e, saved=saved, boundary="periodic", n_pbc=4, warm_start=True)
    torch.cuda.synchronize()
    ra = oracle.forward(dict(w, n_pbc=3), want_phi=True)
    rb = oracle.forward(dict(w, n_pbc=4), phi_init=ra["phi"])
    assert_field_close(J.cpu().numpy(), rb["J"], name="J warm")
    assert_field_close(A.cpu().numpy(), rb["absorbed"], name="absorbed warm")
    # 3 passes then 4 warm-started passes = 7 passes from zero inflow
    J7, _, _ = sw.forward(dag, k, e, boundary="periodic", n_pbc=7)
    assert_field_close(J.cpu().numpy(), J7.cpu().numpy().astype(np.float64), name="J 3+4 vs 7")


@pytest.mark.parametrize("merge,n_pbc,n_scat", [(False, 3, 1), (False, 2, 3), (True, 2, 3)])
def test_warm_start_adjoint_matches_oracle(merge, n_pbc, n_scat):
    """The adjoint of a warm-started call (the first pass's periodic inflow taken
    from the workspace's earlier final pass, held fixed) against the oracle's;
    with several iterations, or merged, the workspace also keeps that inflow for
    the adjoint's recomputation of the first pass."""
    import ctypes
    sw = _sw()
    G = 2
    w = W.small_random(2000, 24, G=G, seed=98 + n_pbc, periodic=True, n_pbc=n_pbc, albedo=0.4,
                       n_scat=n_scat, n_src=4, tau=2.0)
    w = dict(w, merge=merge)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    opts = dict(_opts(w), merge=merge)
    need = sw.sweep_saved_bytes(dag.handle, G, ctypes.byref(sw._fwd_opts(warm_start=True, **opts)))
    saved = torch.empty(need // 4, dtype=torch.float32, device="cuda")
    k0 = k * 1.3  # the earlier run: other opacities
    sw.forward(dag, k0, e, saved=saved, **opts)
    torch.cuda.synchronize()
    warm = oracle.forward(dict(w, kappa=np.asarray(w["kappa"], np.float64) * 1.3), want_phi=True)["phi"]
    J, A, tot, _ = sw.forward(dag, k, e, saved=saved, warm_start=True, **opts)
    rng = np.random.default_rng(15)
    C = len(w["meshes"][0]["cell_volume"])
    gJ = rng.random((C, G)).astype(np.float32)
    gA = rng.random((C, G)).astype(np.float32)
    dk, de = sw.adjoint(dag, k, e, saved, torch.tensor(gJ, device="cuda"),
                        torch.tensor(gA, device="cuda"), warm_start=True, **opts)
    ref = oracle.forward(w, phi_init=warm)
    assert_field_close(J.cpu().numpy(), ref["J"], name="J warm")
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA, phi_init=warm)
    _grad_close(dk.cpu().numpy(), dk_ref)
    _grad_close(de.cpu().numpy(), de_ref)


@pytest.mark.parametrize("tol,n_scat", [(0.25, 2), (0.3, 3)])
def test_pbc_tol_adjoint_matches_oracle(tol, n_scat):
    """pbc_tol ends each iteration's passes once E is below it; the forward keeps
    the pass counts in the workspace and the adjoint runs those passes (the
    counts held fixed), against the oracle's adjoint of the same stopping."""
    sw = _sw()
    G = 1
    w = W.small_random(200, 8, G=G, seed=17, periodic=True, n_pbc=10, n_src=3, albedo=0.4,
                       n_scat=n_scat, tau=2.0)
    w = dict(w, pbc_tol=tol)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    opts = dict(_opts(w), pbc_tol=tol)
    J, A, tot, saved = sw.forward(dag, k, e, save_for_adjoint=True, **opts)
    ref = oracle.forward(w)
    assert_field_close(J.cpu().numpy(), ref["J"], name="J")  # the same passes ran
    rng = np.random.default_rng(16)
    C = len(w["meshes"][0]["cell_volume"])
    gJ = rng.random((C, G)).astype(np.float32)
    gA = rng.random((C, G)).astype(np.float32)
    dk, de = sw.adjoint(dag, k, e, saved, torch.tensor(gJ, device="cuda"),
                        torch.tensor(gA, device="cuda"), **opts)
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA)
    _grad_close(dk.cpu().numpy(), dk_ref)
    _grad_close(de.cpu().numpy(), de_ref)
    # a workspace without the counts (a call without pbc_tol) is refused
    _, _, _, saved0 = sw.forward(dag, k, e, save_for_adjoint=True, **_opts(w))
    with pytest.raises(sw.SweepError, match="INVALID_ARG"):
        sw.adjoint(dag, k, e, saved0, torch.ones_like(k), torch.ones_like(k), **opts)


def test_warm_start_needs_saved():
    sw = _sw()
    w = W.small_random(500, 8, G=1, seed=97, periodic=True)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    with pytest.raises(sw.SweepError, match="INVALID_ARG"):
        sw.forward(dag, k, e, boundary="periodic", warm_start=True)


def test_merged_graph_replays_match_eager():
    sw = _sw()
    w = W.small_random(2000, 24, G=1, seed=98, periodic=True, n_pbc=3, albedo=0.4, n_scat=4)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    J0, A0, t0 = sw.forward(dag, k, e, merge=True, **_opts(w))
    for _ in range(3):
        Jg, Ag, tg = sw.forward(dag, k, e, merge=True, use_graph=True, **_opts(w))
        torch.cuda.synchronize()
        assert torch.equal(Jg, J0) and torch.equal(Ag, A0) and torch.equal(tg, t0)


def test_periodic_error_curve_matches_oracle():
    """E = |j_n - j_{n-1}| / (j_n + j_{n-1}) of the last two passes (eq. relativeErrorPbc),
    max over cells and L1 form, for 2..8 passes: the GPU's curve follows the oracle's
    and falls with every pass after the third."""
    sw = _sw()
    w = W.small_random(3000, 24, G=2, seed=99, periodic=True, n_src=6, tau=2.0)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    curve = []
    for n in range(2, 9):
        _, _, tot = sw.forward(dag, k, e, boundary="periodic", n_pbc=n)
        g = tot.cpu().numpy()[0]
        r = oracle.forward(dict(w, n_pbc=n))["totals"][0]
        assert np.allclose(g[:, 6], r[:, 6], rtol=1e-3, atol=1e-6), n
        assert np.allclose(g[:, 7], r[:, 7], rtol=1e-4, atol=1e-7), n
        curve.append(g[:, 7])
        print("passes %d: E max %s  E L1 %s" % (n, np.array2string(g[:, 6], precision=4),
                                                np.array2string(g[:, 7], precision=4)))
    curve = np.array(curve)
    assert np.all(curve[0] == 1.0)  # the first pass starts from zero inflow
    assert np.all(np.diff(curve[1:], axis=0) < 0)


def test_convergence_threshold_matches_oracle():
    sw = _sw()
    w = W.small_random(3000, 24, G=2, seed=99, periodic=True, n_src=6, tau=2.0)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    # a threshold between the E of 6 and of 7 passes (0.1253 and 0.0707 for group 0,
    # 0.1624 and 0.1135 for group 1): the passes stop after the 7th
    tol = 0.14
    J, A, tot = sw.forward(dag, k, e, boundary="periodic", n_pbc=40, pbc_tol=tol)
    J7, A7, tot7 = sw.forward(dag, k, e, boundary="periodic", n_pbc=7)
    torch.cuda.synchronize()
    assert torch.equal(J, J7) and torch.equal(A, A7)
    assert np.allclose(tot.cpu().numpy(), tot7.cpu().numpy(), rtol=1e-12, atol=0)
    ref = oracle.forward(dict(w, n_pbc=40, pbc_tol=tol))
    assert_field_close(J.cpu().numpy(), ref["J"], name="J")
    assert tot.cpu().numpy()[..., 6].max() < tol
    for bad in (dict(merge=True, n_scat=2, albedo=0.3), dict(use_graph=True)):
        with pytest.raises(sw.SweepError, match="INVALID_ARG"):
            sw.forward(dag, k, e, boundary="periodic", n_pbc=5, pbc_tol=tol, **bad)


def test_merge_without_scattering_keeps_the_nested_workspace():
    """merge only takes effect with several source iterations; with n_scat = 1 the
    forward is the nested order and keeps every pass for the adjoint, so the
    workspace size must include them (regression)."""
    sw = _sw()
    w = W.small_random(1500, 8, G=1, seed=100, periodic=True, n_pbc=3, n_src=4, tau=2.0)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    o = dict(boundary="periodic", n_pbc=3, merge=True)
    assert dag.saved_bytes(1, **o) == dag.saved_bytes(1, boundary="periodic", n_pbc=3)
    J, A, tot, saved = sw.forward(dag, k, e, save_for_adjoint=True, **o)
    gJ = torch.ones_like(k)
    gA = torch.zeros_like(k)
    dk, de = sw.adjoint(dag, k, e, saved, gJ, gA, **o)
    dk_ref, de_ref = oracle.adjoint(w, np.ones((1500, 1)), np.zeros((1500, 1)))
    from tests.test_gpu_parity import _grad_close
    _grad_close(dk.cpu().numpy(), dk_ref)
    _grad_close(de.cpu().numpy(), de_ref)
