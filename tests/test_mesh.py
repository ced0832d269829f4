"""Pins of the synthetic Voronoi meshes (input generator)."""
import os

import numpy as np
import pytest

from synth.mesh import voronoi_mesh, lattice_mesh, morton_order

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def _golden(key):
    for line in open(GOLDEN):
        line = line.split("#")[0].split()
        if len(line) == 2 and line[0] == key:
            return float(line[1])
    raise KeyError(key)


def _owner(m):
    return np.repeat(np.arange(len(m["cell_volume"])), np.diff(m["face_ptr"]))


@pytest.mark.parametrize("periodic", [False, True])
def test_geometry_invariants(periodic):
    rng = np.random.default_rng(7)
    m = voronoi_mesh(rng.random((3000, 3)), periodic=periodic)
    C = 3000
    own = _owner(m)
    assert abs(m["cell_volume"].sum() - 1.0) < 1e-12
    clos = np.zeros((C, 3))
    np.add.at(clos, own, m["face_area"][:, None] * m["face_normal"])
    surf = np.bincount(own, m["face_area"], minlength=C)
    assert np.max(np.linalg.norm(clos, axis=1) / surf) < 1e-12
    assert np.allclose(np.linalg.norm(m["face_normal"], axis=1), 1.0, atol=1e-14)
    tw = m["face_twin"]
    inner = np.nonzero(m["face_nbr"] >= 0)[0]
    assert np.all(tw[inner] >= 0)
    assert np.array_equal(tw[tw[inner]], inner)
    assert np.array_equal(own[tw[inner]], m["face_nbr"][inner])
    assert np.array_equal(m["face_area"][tw[inner]], m["face_area"][inner])
    assert np.array_equal(m["face_normal"][tw[inner]], -m["face_normal"][inner])
    assert np.array_equal(m["face_shift"][tw[inner]], -m["face_shift"][inner])
    # Voronoi normals point from the seed to the neighbour's seed (appendix A)
    d = m["points"][m["face_nbr"][inner]] - m["points"][own[inner]]
    if periodic:
        d -= np.round(d)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    assert np.allclose(d, m["face_normal"][inner], atol=1e-12)
    if periodic:
        assert np.all(m["face_nbr"] >= 0)
    else:
        walls = m["face_nbr"] < 0
        assert abs(m["face_area"][walls].sum() - 6.0) < 1e-10


def test_mean_neighbour_count_matches_paper():
    """Mean neighbours of a 3D Poisson-Voronoi cell (the 15.54 quoted in sec. 2.6)."""
    rng = np.random.default_rng(8)
    m = voronoi_mesh(rng.random((40000, 3)), periodic=True)
    mean = len(m["face_nbr"]) / len(m["cell_volume"])
    assert abs(mean - _golden("mean_voronoi_neighbours")) < 0.05
    assert abs(mean / 2 - _golden("mean_downwind_dependencies")) < 0.05


def test_matches_qhull_box_clipped():
    """Face areas and volumes agree with scipy's Qhull Voronoi of the seeds mirrored in the walls."""
    from scipy.spatial import ConvexHull, Voronoi
    rng = np.random.default_rng(9)
    n = 300
    m = voronoi_mesh(rng.random((n, 3)), periodic=False)
    p = m["points"]
    allp = [p]
    for ax in range(3):
        for wall in (0.0, 1.0):
            q = p.copy()
            q[:, ax] = 2 * wall - q[:, ax]
            allp.append(q)
    vor = Voronoi(np.concatenate(allp))
    own = _owner(m)
    ours = {}
    for f in np.nonzero(m["face_nbr"] >= 0)[0]:
        ours[(int(own[f]), int(m["face_nbr"][f]))] = m["face_area"][f]
    seen = 0
    for (a, b), rv in zip(vor.ridge_points, vor.ridge_vertices):
        if a >= n or b >= n or -1 in rv:
            continue
        verts = vor.vertices[rv]
        nrm = p[b] - p[a]
        nrm /= np.linalg.norm(nrm)
        e1 = np.cross(nrm, [1.0, 0, 0] if abs(nrm[0]) < 0.9 else [0, 1.0, 0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(nrm, e1)
        xy = np.stack([verts @ e1, verts @ e2], axis=1)
        area = ConvexHull(xy).volume if len(verts) >= 3 else 0.0
        key = (a, b)
        if area < 1e-12:
            continue
        assert key in ours and (b, a) in ours
        assert abs(ours[key] - area) < 1e-9 * max(area, 1e-6)
        seen += 1
    assert seen == len(ours) // 2 or abs(seen - len(ours) // 2) <= 2
    for c in rng.choice(n, 20, replace=False):
        reg = vor.regions[vor.point_region[c]]
        vol = ConvexHull(vor.vertices[reg]).volume
        assert abs(vol - m["cell_volume"][c]) < 1e-10


def test_lattice_mesh():
    m = lattice_mesh(4, periodic=False)
    assert len(m["cell_volume"]) == 64 and np.allclose(m["cell_volume"].sum(), 1)
    assert np.count_nonzero(m["face_nbr"] < 0) == 6 * 16
    mp = lattice_mesh(4, periodic=True)
    tw = mp["face_twin"]
    assert np.array_equal(tw[tw], np.arange(len(tw)))
    assert np.count_nonzero(mp["face_shift"]) == 6 * 16


def test_morton_order_is_permutation():
    rng = np.random.default_rng(10)
    p = rng.random((1000, 3))
    o = morton_order(p)
    assert np.array_equal(np.sort(o), np.arange(1000))
