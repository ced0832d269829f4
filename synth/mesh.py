"""Seeded synthetic Voronoi meshes for the sweep workloads.

A mesh is a dict of numpy arrays describing a Voronoi grid in the unit box
(the grid of the paper's section 2.1: cells with face areas A_i and unit face
normals n_i, section 2.6; normals n = (p' - p)/|p' - p| as in appendix A):

    points       f64 [C,3]   generating points (Morton order)
    face_ptr     i64 [C+1]   CSR offsets of each cell's half-faces
    face_nbr     i32 [F]     neighbour cell, -1 for a vacuum box wall
    face_twin    i32 [F]     index of the matching half-face in the neighbour, -1 for walls
    face_shift   i8  [F]     periodic image code of the neighbour (0 = none)
    face_area    f64 [F]
    face_normal  f64 [F,3]   unit normal, outward from the owner
    cell_volume  f64 [C]
    periodic     bool

Twin half-faces carry bit-identical areas and exactly negated normals (taken
from the canonical side: owner < neighbour, or the positive image for a cell
facing its own image).  Nothing here computes any part of the transport sweep.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "voronoi.cpp")
_LIB = os.path.join(_HERE, "libvoro.so")
_lib = None


def build_lib(force: bool = False) -> str:
    """Compile the Voronoi builder (g++, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_lib()
        lib = ctypes.CDLL(_LIB)
        lib.voro_build.restype = ctypes.c_void_p
        lib.voro_build.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p]
        lib.voro_rebuild.restype = None
        lib.voro_rebuild.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p]
        lib.voro_counts.restype = ctypes.c_int64
        lib.voro_counts.argtypes = [ctypes.c_void_p]
        lib.voro_fetch.restype = None
        lib.voro_fetch.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6
        lib.voro_free.restype = None
        lib.voro_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def morton_order(points: np.ndarray) -> np.ndarray:
    """Permutation sorting points along a 3D Morton (Z-order) curve."""
    q = np.clip((points * (1 << 21)).astype(np.int64), 0, (1 << 21) - 1).astype(np.uint64)

    def spread(v):
        v = v & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v

    code = spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1)) | (spread(q[:, 2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


def _candidates(tree, queries: np.ndarray, n: int, k: int):
    k = min(k, n)
    _, idx = tree.query(queries, k=k, workers=-1)
    idx = np.asarray(idx, dtype=np.int32).reshape(len(queries), k)
    return np.ascontiguousarray(idx)


def _raw_build(points: np.ndarray, periodic: bool, k0: int = 48):
    """Clip every cell against its k0 nearest seeds; cells whose candidates ran
    out before the security radius are rebuilt alone with twice as many."""
    from scipy.spatial import cKDTree
    lib = _load()
    n = len(points)
    pts = np.ascontiguousarray(points, dtype=np.float64)
    tree = cKDTree(pts, boxsize=1.0 if periodic else None)
    k = min(k0, n)
    status = np.zeros(n, dtype=np.int32)
    h = lib.voro_build(n, _ptr(pts), int(periodic), k, _ptr(_candidates(tree, pts, n, k)),
                       _ptr(status))
    bad = np.nonzero(status == 1)[0].astype(np.int32)
    while len(bad) and k < n:
        k = min(2 * k, n)
        cand = _candidates(tree, pts[bad], n, k)
        st = np.zeros(len(bad), dtype=np.int32)
        lib.voro_rebuild(h, len(bad), _ptr(bad), _ptr(pts), int(periodic), k, _ptr(cand), _ptr(st))
        status[bad] = st
        bad = bad[st == 1]
    if (status == 2).any():
        lib.voro_free(h)
        raise RuntimeError("degenerate Voronoi cell")
    if (status == 3).any():
        lib.voro_free(h)
        raise RuntimeError("periodic mesh too coarse for minimum-image neighbours")
    nf = lib.voro_counts(h)
    face_ptr = np.empty(n + 1, np.int64)
    nbr = np.empty(nf, np.int32)
    shift = np.empty(nf, np.int8)
    area = np.empty(nf, np.float64)
    normal = np.empty((nf, 3), np.float64)
    volume = np.empty(n, np.float64)
    lib.voro_fetch(h, _ptr(face_ptr), _ptr(nbr), _ptr(shift), _ptr(area), _ptr(normal), _ptr(volume))
    lib.voro_free(h)
    return face_ptr, nbr, shift, area, normal, volume


def _pair_faces(face_ptr, nbr, shift, area, normal, n):
    """Match every half-face with its twin; drop unmatched slivers; make twins exact."""
    owner = np.repeat(np.arange(n, dtype=np.int64), np.diff(face_ptr))
    s = shift.astype(np.int64)
    interior = nbr >= 0
    nb = nbr.astype(np.int64)
    key = np.where(interior, (owner * n + nb) * 27 + (s + 13), -1)
    tkey = np.where(interior, (nb * n + owner) * 27 + (-s + 13), -2)
    order = np.argsort(key, kind="stable")
    sk = key[order]
    pos = np.searchsorted(sk, tkey)
    pos = np.clip(pos, 0, len(sk) - 1)
    found = sk[pos] == tkey
    twin = np.where(found, order[pos], -1)
    keep = (~interior) | found
    # re-index after dropping unmatched interior half-faces
    new_index = np.cumsum(keep) - 1
    counts = np.bincount(owner[keep], minlength=n)
    new_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=new_ptr[1:])
    idx = np.nonzero(keep)[0]
    nbr2 = nbr[idx].copy()
    shift2 = shift[idx].copy()
    area2 = area[idx].copy()
    normal2 = normal[idx].copy()
    twin2 = np.where(twin[idx] >= 0, new_index[np.maximum(twin[idx], 0)], -1).astype(np.int32)
    # canonical side: owner < nbr, or own image with positive code
    own2 = owner[idx]
    canon = (nbr2 >= 0) & ((own2 < nbr2) | ((own2 == nbr2) & (shift2 > 0)))
    ci = np.nonzero(canon)[0]
    ti = twin2[ci]
    area2[ti] = area2[ci]
    normal2[ti] = -normal2[ci]
    return new_ptr, nbr2, twin2, shift2, area2, normal2


def voronoi_mesh(points: np.ndarray, periodic: bool = False, morton: bool = True) -> dict:
    """Voronoi grid of `points` in the unit box, box-clipped or periodic."""
    points = np.asarray(points, dtype=np.float64)
    if periodic:
        points = np.mod(points, 1.0)
        points[points >= 1.0] = 0.0
    if morton:
        points = points[morton_order(points)]
    n = len(points)
    face_ptr, nbr, shift, area, normal, volume = _raw_build(points, periodic)
    face_ptr, nbr, twin, shift, area, normal = _pair_faces(face_ptr, nbr, shift, area, normal, n)
    return dict(points=np.ascontiguousarray(points), face_ptr=face_ptr, face_nbr=nbr,
                face_twin=twin, face_shift=shift, face_area=area,
                face_normal=np.ascontiguousarray(normal), cell_volume=volume,
                periodic=bool(periodic))


def lattice_mesh(n: int, periodic: bool = False) -> dict:
    """Analytic cubic-lattice grid of n^3 unit-box cells (cell (i,j,k) = i + n*(j + n*k)).

    Faces are ordered -x, +x, -y, +y, -z, +z; walls (vacuum) have nbr -1.
    """
    h = 1.0 / n
    cid = np.arange(n ** 3, dtype=np.int64)
    i, j, k = cid % n, (cid // n) % n, cid // (n * n)
    C = n ** 3
    pts = np.stack([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h], axis=1)
    dirs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    nbr = np.empty((C, 6), np.int64)
    shift = np.zeros((C, 6), np.int8)
    normal = np.zeros((C, 6, 3))
    for f, (dx, dy, dz) in enumerate(dirs):
        ni, nj, nk = i + dx, j + dy, k + dz
        sx = np.where(ni < 0, -1, np.where(ni >= n, 1, 0))
        sy = np.where(nj < 0, -1, np.where(nj >= n, 1, 0))
        sz = np.where(nk < 0, -1, np.where(nk >= n, 1, 0))
        out = (sx != 0) | (sy != 0) | (sz != 0)
        ni, nj, nk = ni % n, nj % n, nk % n
        nid = ni + n * (nj + n * nk)
        if periodic:
            nbr[:, f] = nid
            shift[:, f] = ((sx + 1) * 9 + (sy + 1) * 3 + (sz + 1) - 13).astype(np.int8)
        else:
            nbr[:, f] = np.where(out, -1, nid)
        normal[:, f] = (dx, dy, dz)
    # twin of face f is the opposite face of the neighbour
    opp = np.array([1, 0, 3, 2, 5, 4])
    twin = np.where(nbr >= 0, nbr * 6 + opp[None, :], -1)
    return dict(points=pts, face_ptr=np.arange(0, 6 * C + 1, 6, dtype=np.int64),
                face_nbr=nbr.reshape(-1).astype(np.int32), face_twin=twin.reshape(-1).astype(np.int32),
                face_shift=shift.reshape(-1), face_area=np.full(6 * C, h * h),
                face_normal=normal.reshape(-1, 3).copy(), cell_volume=np.full(C, h ** 3),
                periodic=bool(periodic))


def mesh_stats(mesh: dict) -> dict:
    C = len(mesh["cell_volume"])
    F = len(mesh["face_nbr"])
    v = mesh["cell_volume"]
    return dict(n_cells=C, n_half_faces=F, faces_per_cell=F / C,
                vol_p1=float(np.percentile(v, 1)), vol_p99=float(np.percentile(v, 99)),
                vol_span=float(v.max() / v.min()))


def complete_graph_mesh(n: int, seed: int = 0) -> dict:
    """Combinatorial test mesh: every cell shares a face with every other cell
    (plus six vacuum walls), face normals n_ij = (p_j - p_i)/|p_j - p_i| for
    random points p, so every direction's graph stays acyclic (the projection
    on the direction orders it).  Areas and volumes are random; twins carry the
    same area and the negated normal.  Cells have n + 5 faces: far more than a
    Voronoi cell, for the code paths of cells with many faces."""
    rng = np.random.default_rng(np.random.SeedSequence([2207, 12848, 900, seed]))
    p = rng.random((n, 3))
    area_ij = rng.uniform(0.2, 1.0, size=(n, n))
    area_ij = np.triu(area_ij, 1)
    area_ij = area_ij + area_ij.T
    walls = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], np.float64)
    nf = n - 1 + 6
    face_ptr = np.arange(n + 1, dtype=np.int64) * nf
    nbr = np.empty((n, nf), np.int32)
    area = np.empty((n, nf))
    normal = np.empty((n, nf, 3))
    slot = np.empty((n, n), np.int64)  # face index of neighbour j in cell c
    for c in range(n):
        others = [j for j in range(n) if j != c]
        nbr[c, :n - 1] = others
        nbr[c, n - 1:] = -1
        for k, j in enumerate(others):
            slot[c, j] = c * nf + k
            if c < j:
                d = p[j] - p[c]
                normal[c, k] = d / np.linalg.norm(d)
            area[c, k] = area_ij[c, j]
        area[c, n - 1:] = rng.uniform(0.5, 1.0, size=6)
        normal[c, n - 1:] = walls
    for c in range(n):  # twins: exact negation of the canonical side
        for k, j in enumerate(nbr[c, :n - 1]):
            if c > j:
                normal[c, k] = -normal[j, slot[j, c] - j * nf]
    twin = np.full((n, nf), -1, np.int32)
    for c in range(n):
        for k, j in enumerate(nbr[c, :n - 1]):
            twin[c, k] = slot[j, c]
    return dict(points=p, face_ptr=face_ptr, face_nbr=nbr.reshape(-1), face_twin=twin.reshape(-1),
                face_shift=np.zeros(n * nf, np.int8), face_area=area.reshape(-1),
                face_normal=np.ascontiguousarray(normal.reshape(-1, 3)),
                cell_volume=rng.uniform(0.05, 0.2, size=n), periodic=False)
