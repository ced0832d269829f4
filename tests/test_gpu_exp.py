"""GPU parity of the exponential cell law (transmission e^{-tau}, tau = kappa V / Aperp)
against the FP64 oracle, with the tolerances of the upwind law's parity tests."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from synth import workloads as W  # noqa: E402
from synth.directions import direction_set  # noqa: E402
from tests.test_gpu_parity import _dev, _grad_close, _opts, _sw, check_forward, run_gpu  # noqa: E402


def _exp(w):
    return dict(w, law="exp")


def test_exp_forward_c1():
    check_forward(_exp(W.c1_plain_small()))


@pytest.mark.parametrize("G", [1, 4])
def test_exp_forward_groups_multimesh(G):
    check_forward(_exp(W.small_random(1500, 24, G=G, seed=70 + G, n_meshes=3, n_src=5)))


def test_exp_forward_periodic_and_scattering():
    w = _exp(W.small_random(2000, 8, G=2, seed=73, periodic=True, n_pbc=3, albedo=0.3, n_scat=3))
    dag, J, A, tot, ref = check_forward(w)
    assert np.allclose(tot[..., 6], ref["totals"][..., 6], rtol=1e-4, atol=1e-6)


def test_exp_forward_scattering_plain_form():
    w = _exp(W.small_random(1200, 24, G=2, seed=74, n_src=4, albedo=0.5, n_scat=4))
    check_forward(w, form="plain")


def test_exp_thick_and_thin_cells():
    # optical depths beyond the cap of 40 (the transmission floor) next to kappa = 0
    w = _exp(W.small_random(3000, 24, G=2, seed=75, n_src=8))
    k = np.array(w["kappa"], np.float64)
    rng = np.random.default_rng(7)
    k[rng.choice(3000, 150, replace=False)] *= 1e4
    k[rng.choice(3000, 150, replace=False)] = 0.0
    w["kappa"] = k
    check_forward(w)


def test_exp_equals_upwind_without_absorption():
    w = W.small_random(800, 24, G=2, seed=76, n_src=4)
    w["kappa"] = np.zeros_like(w["kappa"])
    _, J0, A0, t0 = run_gpu(w)
    _, J1, A1, t1 = run_gpu(_exp(w))
    assert np.array_equal(J0, J1) and np.array_equal(t0, t1)


def test_exp_lattice_beam_is_exponential():
    n = 12
    row = [m + n * (5 + n * 7) for m in range(n)]
    w = _exp(W.lattice_workload(n, np.array([[1.0, 0.0, 0.0]]), 2.0, [row[0]], [1.0]))
    dag, J, A, tot, ref = check_forward(w)
    kap = float(np.float32(2.0))
    h = 1.0 / n
    # each cell passes on exactly e^{-kappa h} of what enters it
    ratio = J[row[1:], 0].astype(np.float64) / J[row[:-1], 0]
    assert np.allclose(ratio, np.exp(-kap * h), rtol=1e-5)
    assert abs(tot[0, 0, 2] - np.exp(-kap)) <= 1e-5 * np.exp(-kap)


@pytest.mark.parametrize("albedo,n_scat,G", [(0.0, 1, 1), (0.0, 1, 3), (0.5, 4, 2)])
def test_exp_adjoint_matches_oracle(albedo, n_scat, G):
    sw = _sw()
    w = _exp(W.small_random(2000, 24, G=G, seed=80 + n_scat, n_src=4, albedo=albedo,
                            n_scat=n_scat, n_meshes=2))
    rng = np.random.default_rng(8)
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


def test_exp_adjoint_thin_and_capped_cells():
    sw = _sw()
    w = _exp(W.small_random(1500, 8, G=1, seed=83, n_src=4, albedo=0.3, n_scat=2))
    k = np.array(w["kappa"], np.float64)
    rng = np.random.default_rng(9)
    k[rng.choice(1500, 60, replace=False)] *= 1e4
    k[rng.choice(1500, 60, replace=False)] = 3e-3
    w["kappa"] = k.astype(np.float32)
    C = 1500
    gJ = rng.random((C, 1)).astype(np.float32)
    gA = rng.random((C, 1)).astype(np.float32)
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    kk, e = _dev(w)
    J, A, tot, saved = sw.forward(dag, kk, e, save_for_adjoint=True, **_opts(w))
    dk, de = sw.adjoint(dag, kk, e, saved, torch.tensor(gJ, device="cuda"),
                        torch.tensor(gA, device="cuda"), **_opts(w))
    _grad_close(dk.cpu().numpy(), dk_ref)
    _grad_close(de.cpu().numpy(), de_ref)


def test_exp_autograd_function_and_graph():
    sw = _sw()
    w = _exp(W.small_random(1500, 24, G=1, seed=84, n_src=3))
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    k.requires_grad_(True)
    e.requires_grad_(True)
    J, A, tot = sw.SweepFunction.apply(k, e, dag, dict(_opts(w), use_graph=True))
    loss = A.sum() / (4 * np.pi)
    loss.backward()
    gJ, gA = oracle.absorbed_loss_grads(w)
    dk_ref, de_ref = oracle.adjoint(w, gJ, gA)
    _grad_close(k.grad.cpu().numpy(), dk_ref)
    _grad_close(e.grad.cpu().numpy(), de_ref)
    # the two laws keep separate captured graphs
    J_up, _, _ = sw.forward(dag, k.detach(), e.detach(), use_graph=True,
                            **dict(_opts(w), law="upwind"))
    J_ex, _, _ = sw.forward(dag, k.detach(), e.detach(), use_graph=True, **_opts(w))
    torch.cuda.synchronize()
    assert np.array_equal(J_ex.cpu().numpy(), J.detach().cpu().numpy())
    assert not np.array_equal(J_up.cpu().numpy(), J_ex.cpu().numpy())


def test_exp_single_cell_closed_form():
    dirs = direction_set(24)
    w = _exp(W.lattice_workload(1, dirs, 0.7, [0], [3.0]))
    dag, J, A, tot, ref = check_forward(w)
    ap = np.abs(dirs).sum(axis=1)
    kap = float(np.float32(0.7))
    avg = (3.0 / 24) * (1.0 - np.exp(-kap / ap)) / kap
    assert abs(J[0, 0] - avg.sum() / (4 * np.pi)) <= 1e-5 * J[0, 0]


def test_unknown_law_is_rejected():
    import ctypes
    sw = _sw()
    w = W.small_random(200, 8, seed=85)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    k, e = _dev(w)
    o = sw._fwd_opts()
    o.law = 7
    G = k.shape[1]
    J = torch.empty_like(k)
    A = torch.empty_like(k)
    tot = torch.empty((1, G, 8), dtype=torch.float64, device="cuda")
    st = sw.sweep_forward(dag.handle, G, k.data_ptr(), e.data_ptr(), ctypes.byref(o), J.data_ptr(),
                          A.data_ptr(), tot.data_ptr(), None, 0, None)
    assert st == -1  # SWEEP_ERR_INVALID_ARG
    assert "law" in sw.sweep_last_error()
