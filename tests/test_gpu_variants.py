"""GPU parity of the code paths that only some sizes take, each forced on inputs the
oracle checks element by element (through the C ABI):

- the level computation with its per-cell counters in global memory (taken
  above ~290 K cells per mesh) against the LDS counters and the oracle's levels;
- the persistent sweep in which one workgroup sweeps several (mesh, direction)
  units in turn (taken when the units outnumber the resident workgroups), with a
  small grid forced, and with the 64 uneven meshes of the scattering workload
  (1,536 units) at reduced cell counts;
- levels wider than the workgroup, cut into several steps (small workgroups);
- rings too small to hold three steps, where values that could not be prefetched
  are read from global memory at solve time;
- every packing of the groups into work items (1 to 4 groups per workgroup),
  which must agree bit for bit, and the periodic adjoint, which must not depend
  on the run or the grid.

Tolerances as in test_gpu_parity: graphs bit-exact, J and absorbed within 1e-5
relative (elementwise above 1e-20 of the maximum, and in L1), gradients within
1e-5 in relative L2 and elementwise 1e-4 relative + 1e-6 of the largest."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from synth import workloads as W  # noqa: E402

REL = 1e-5
INV4PI = 1.0 / (4.0 * np.pi)


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


def field_close(gpu, ref, rel=REL, floor=1e-20, name="field"):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert np.all(np.isfinite(gpu)), name
    big = np.abs(ref) >= floor * np.abs(ref).max()
    err = np.abs(gpu - ref)
    worst = (err[big] / np.abs(ref[big])).max()
    l1 = err.sum() / np.abs(ref).sum()
    print("%s: max rel %.3e  rel L1 %.3e" % (name, worst, l1))
    assert worst <= rel and l1 <= rel, name


def grad_close(g, r, name):
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    l2 = np.linalg.norm(g - r) / np.linalg.norm(r)
    excess = np.abs(g - r) - (1e-4 * np.abs(r) + 1e-6 * np.abs(r).max())
    print("%s: rel L2 %.3e" % (name, l2))
    assert l2 <= 1e-5 and excess.max() <= 0.0, name


def gpu_run(w, adjoint=True, build=None, **kw):
    sw = _sw()
    dag = sw.build_dag(w["meshes"], w["dirs"], **(build or {}))
    k, e = _dev(w)
    out = {}
    J, A, tot, saved = sw.forward(dag, k, e, save_for_adjoint=True, **_opts(w), **kw)
    if adjoint:
        gJ = torch.zeros_like(k)
        gA = torch.full_like(k, INV4PI)
        dk, de = sw.adjoint(dag, k, e, saved, gJ, gA, **_opts(w), **kw)
        out["dk"], out["de"] = dk.cpu().numpy(), de.cpu().numpy()
    torch.cuda.synchronize()
    out["J"], out["A"], out["tot"] = J.cpu().numpy(), A.cpu().numpy(), tot.cpu().numpy()
    out["info"] = dag.info()
    out["dag"] = dag
    return out


def check_against_oracle(w, g, adjoint=True):
    ref = oracle.forward(w)
    field_close(g["J"], ref["J"], name="J")
    field_close(g["A"], ref["absorbed"], name="absorbed")
    if adjoint:
        gJ, gA = oracle.absorbed_loss_grads(w)
        dk, de = oracle.adjoint(w, gJ, gA)
        grad_close(g["dk"], dk, "dL/dkappa")
        grad_close(g["de"], de, "dL/demission")


def dag_matches_oracle(dag, w):
    lv, od, ind = dag.export()
    for m, mesh in enumerate(w["meshes"]):
        rl, ro, ri, rd = oracle.build_dag(mesh, w["dirs"])
        assert np.array_equal(dag.split(lv)[m], rl)
        assert np.array_equal(dag.split(od)[m], ro)
        assert np.array_equal(dag.split(ind)[m], ri)
        assert np.array_equal(dag.depths()[m], rd)


@pytest.mark.parametrize("case", ["multi", "periodic", "many_faces"])
def test_global_kahn_counters_match_oracle(case):
    """The level computation with counters in global memory (the path of meshes
    above ~290 K cells), forced on small meshes: levels, order and counts
    bit-exact, and the sweeps built on them against the oracle."""
    sw = _sw()
    if case == "multi":
        w = W.small_random(1500, 24, seed=31, n_meshes=3)
    elif case == "periodic":
        w = W.small_random(1200, 48, seed=32, periodic=True, n_pbc=3)
    else:
        w = W.many_faces(60, 24, seed=3)
    for mode in ("global", "lds"):
        dag = sw.build_dag(w["meshes"], w["dirs"], kahn_counters=mode)
        assert dag.info()["kahn_lds_counters"] == (1 if mode == "lds" else 0)
        dag_matches_oracle(dag, w)
        dag.close()
    g = gpu_run(w, build=dict(kahn_counters="global"))
    assert g["info"]["kahn_lds_counters"] == 0
    check_against_oracle(w, g)


def test_lds_counters_forced_on_a_small_mesh():
    sw = _sw()
    w = W.small_random(400, 8, seed=33)
    dag = sw.build_dag(w["meshes"], w["dirs"], kahn_counters="lds")
    assert dag.info()["kahn_lds_counters"] == 1
    dag.close()


@pytest.mark.parametrize("grid", [1, 5])
def test_persistent_workgroups_take_several_units(grid):
    """Fewer persistent workgroups than units: each workgroup sweeps several
    (mesh, direction) units one after another (forward and adjoint, with
    scattering iterations), against the oracle and bit for bit against the
    default grid."""
    w = W.small_random(900, 24, seed=34, n_meshes=4, albedo=0.4, n_scat=3)
    g = gpu_run(w, grid=grid)
    d = gpu_run(w)
    assert np.array_equal(g["J"], d["J"]) and np.array_equal(g["dk"], d["dk"])
    check_against_oracle(w, g)


def test_c5_all_meshes_reduced_sizes():
    """The uneven-mesh scattering workload with all 64 meshes (64 x 24 = 1,536
    units against 256 resident workgroups, so every workgroup sweeps several
    units per pass) at 4,096-16,384 cells per mesh, 5 source iterations:
    forward and adjoint against the oracle."""
    w = W.c5_uneven_scatter(n_meshes=64, lo=4096, hi=16384, n_scat=5)
    g = gpu_run(w)
    assert g["info"]["n_meshes"] == 64 and 64 * 24 > 256
    check_against_oracle(w, g)


@pytest.mark.parametrize("block", [256, 512])
def test_wide_levels_cut_into_steps(block):
    """The 64^3 jittered lattice has levels of up to 563 tasks (24 directions):
    with 256- or 512-thread workgroups they are cut into several steps of one
    level each."""
    sw = _sw()
    w = W.c2_plain_scale(n_side=64, D=24, n_src=20)
    dag = sw.build_dag(w["meshes"], w["dirs"])
    lv = dag.split(dag.export()[0])[0]
    widest = max(np.bincount(lv[d]).max() for d in range(lv.shape[0]))
    assert widest > block  # some level wider than the workgroup
    dag.close()
    g = gpu_run(w, block=block)
    check_against_oracle(w, g)


@pytest.mark.parametrize("G,pack", [(1, 0), (4, 4), (4, 2)])
def test_small_ring_reads_unprefetched_values(G, pack):
    """A ring of 64 slots holds less than three steps, so upwind results that are
    outside the ring but not yet final when the values are prefetched are read
    from global memory when the task is solved."""
    w = W.small_random(2500, 24, G=G, seed=35, periodic=True, n_pbc=2)
    g = gpu_run(w, ring=64, block=256, pack=pack)
    d = gpu_run(w)
    check_against_oracle(w, g)
    # the arithmetic does not depend on where a value came from
    assert np.array_equal(g["J"], d["J"]) and np.array_equal(g["dk"], d["dk"])


def test_periodic_adjoint_is_deterministic():
    """The adjoint of the periodic passes takes the later pass's lambda through the
    periodic outflow entries of the downwind rows inside the sweep (no atomics):
    repeated runs and different grids give identical gradients."""
    w = W.small_random(2500, 24, G=2, seed=37, periodic=True, n_pbc=4, albedo=0.2, n_scat=2)
    a = gpu_run(w)
    b = gpu_run(w)
    c = gpu_run(w, grid=3)
    for k in ("dk", "de"):
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k
    check_against_oracle(w, a)


def test_packings_agree_bit_for_bit():
    """Four groups swept as 4 x 1, 2 x 2, 3 + 1 and 1 x 4 packed groups per work
    item (periodic passes, scattering, forward and adjoint): identical results,
    and the oracle's."""
    w = W.small_random(3000, 24, G=4, seed=36, periodic=True, n_pbc=3, albedo=0.3, n_scat=2)
    runs = {p: gpu_run(w, pack=p) for p in (1, 2, 3, 4)}
    for p in (2, 3, 4):
        for k in ("J", "A", "dk", "de"):
            assert np.array_equal(runs[p][k], runs[1][k]), (p, k)
    check_against_oracle(w, runs[2])
    sw = _sw()
    with pytest.raises(sw.SweepError, match="INVALID_ARG"):
        gpu_run(w, pack=5)


def test_c3_recipe_full_size_on_eleven_directions():
    """The clustered periodic mesh at its full 2,097,152 cells with the first 11
    of its 84 directions, 4 groups and 3 periodic passes: the graphs (levels
    computed with counters in global memory: the mesh does not fit LDS) bit-exact
    against the oracle, J and absorbed element by element, and the adjoint of
    the absorbed-photon loss through the periodic passes."""
    sw = _sw()
    w = W.c3_batched_groups()
    w = dict(w, dirs=np.ascontiguousarray(w["dirs"][:11]))
    # two groups per work item, as the full 84 directions take by default
    g = gpu_run(w, pack=2)
    assert g["info"]["kahn_lds_counters"] == 0
    assert g["info"]["max_depth"] > 2700
    dag_matches_oracle(g["dag"], w)
    check_against_oracle(w, g)
    lhs = g["tot"][..., 0] + g["tot"][..., 3] + g["tot"][..., 5]
    rhs = g["tot"][..., 1] + g["tot"][..., 2] + g["tot"][..., 4]
    assert np.all(np.abs(lhs - rhs) <= 1e-6 * g["tot"][..., 0])
    g["dag"].close()
    del sw
