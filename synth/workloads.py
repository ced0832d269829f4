"""Seeded synthetic workloads shaped like the paper's test runs.

The paper sweeps Arepo Voronoi meshes of 32^3..512^3 cells with 84 directions and
one frequency bin; none of its meshes are available, so these seeded stand-ins
are used instead.  Each workload is a dict:

    name, meshes (list of mesh dicts), dirs f64 [D,3], G,
    kappa f32 [C_total, G]    extinction coefficient per cell and group
    emission f32 [C_total, G] isotropic source luminosity per cell and group (photons/s)
    boundary 'vacuum'|'periodic', n_pbc, albedo, n_scat
    sources  i64 [n_src] (global cell ids)

Per-cell arrays are concatenated over meshes (global id = mesh offset + local id)
and stored cell-major with the groups contiguous.  kappa and emission are rounded
to FP32 once here, so every consumer solves the identical problem.

Random streams: np.random.SeedSequence([2207, 12848, k]) for workload k, with
spawned children in the order positions, kappa, sources, mesh sizes.
"""
from __future__ import annotations

import numpy as np

from .directions import direction_set
from .mesh import voronoi_mesh, lattice_mesh


def _streams(k: int, extra: int = 0):
    ss = np.random.SeedSequence([2207, 12848, k] + ([extra] if extra else []))
    return [np.random.default_rng(s) for s in ss.spawn(4)]


# ----------------------------------------------------------------------------- meshes
def uniform_mesh(n: int, rng, periodic: bool = False) -> dict:
    return voronoi_mesh(rng.random((n, 3)), periodic=periodic)


def jittered_lattice_mesh(n_side: int, rng, jitter: float = 0.3, periodic: bool = False) -> dict:
    h = 1.0 / n_side
    g = (np.arange(n_side) + 0.5) * h
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    p = p + rng.uniform(-jitter, jitter, size=p.shape) * h
    return voronoi_mesh(p, periodic=periodic)


def lognormal_density_grid(n_modes: int, sigma: float, rng) -> np.ndarray:
    """rho = exp(sigma*g - sigma) on an n_modes^3 grid, g i.i.d. N(0,1) (white spectrum)."""
    g = rng.standard_normal((n_modes, n_modes, n_modes))
    return np.exp(sigma * g - sigma)


def clustered_points(n: int, rho: np.ndarray, rng) -> np.ndarray:
    m = rho.shape[0]
    p = rho.reshape(-1) / rho.sum()
    cell = rng.choice(m ** 3, size=n, p=p)
    i, j, k = np.unravel_index(cell, rho.shape)
    base = np.stack([i, j, k], axis=1).astype(np.float64)
    return (base + rng.random((n, 3))) / m


def density_at(points: np.ndarray, rho: np.ndarray) -> np.ndarray:
    m = rho.shape[0]
    idx = np.clip((points * m).astype(np.int64), 0, m - 1)
    return rho[idx[:, 0], idx[:, 1], idx[:, 2]]


# ----------------------------------------------------------------------------- fields
def scale_to_mean_tau(kappa: np.ndarray, volume: np.ndarray, tau: float) -> np.ndarray:
    """Scale so that sum(kappa V)/sum(V) = tau (unit box: mean optical depth across it)."""
    return kappa * (tau * volume.sum() / (kappa * volume).sum())


def lognormal_kappa(volume: np.ndarray, rng, sigma: float = 1.0, tau: float = 10.0) -> np.ndarray:
    return scale_to_mean_tau(np.exp(sigma * rng.standard_normal(len(volume))), volume, tau)


def point_sources(n_cells: int, n_src: int, rng, lo: float = -2.0, hi: float = 2.0):
    cells = rng.choice(n_cells, size=min(n_src, n_cells), replace=False)
    lum = 10.0 ** rng.uniform(lo, hi, size=len(cells))
    return np.sort(cells), lum[np.argsort(cells)]


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _workload(name, meshes, D, kappa, emission, sources, boundary="vacuum", n_pbc=1,
              albedo=0.0, n_scat=1):
    kappa = np.asarray(kappa)
    emission = np.asarray(emission)
    if kappa.ndim == 1:
        kappa = kappa[:, None]
    if emission.ndim == 1:
        emission = emission[:, None]
    return dict(name=name, meshes=meshes, dirs=direction_set(D), G=kappa.shape[1],
                kappa=_f32(kappa), emission=_f32(emission), boundary=boundary,
                n_pbc=int(n_pbc), albedo=float(albedo), n_scat=int(n_scat),
                sources=np.asarray(sources, dtype=np.int64))


# ----------------------------------------------------------------------------- configs
def c1_plain_small(n_cells: int = 4096, D: int = 8, tau: float = 5.0) -> dict:
    """4,096 uniform seeds, vacuum, octant diagonals, uniform kappa (box optical depth 5),
    one source of luminosity 1 in the cell nearest the box centre."""
    r_pos, _, _, _ = _streams(1)
    mesh = uniform_mesh(n_cells, r_pos)
    C = len(mesh["cell_volume"])
    d2 = ((mesh["points"] - 0.5) ** 2).sum(axis=1)
    src = int(np.argmin(d2))
    em = np.zeros(C)
    em[src] = 1.0
    return _workload("c1_plain_small", [mesh], D, np.full(C, tau), em, [src])


def c2_plain_scale(n_side: int = 64, D: int = 84, n_src: int = 100, tau: float = 10.0,
                   k: int = 2) -> dict:
    """64^3 lattice jittered by +-0.3 spacing, vacuum, 84 Fibonacci directions, one group,
    100 sources log-uniform in [1e-2, 1e2], lognormal kappa (sigma 1) at mean optical depth 10."""
    r_pos, r_kap, r_src, _ = _streams(k)
    mesh = jittered_lattice_mesh(n_side, r_pos)
    C = len(mesh["cell_volume"])
    kappa = lognormal_kappa(mesh["cell_volume"], r_kap, 1.0, tau)
    cells, lum = point_sources(C, n_src, r_src)
    em = np.zeros(C)
    em[cells] = lum
    return _workload("c2_plain_scale", [mesh], D, kappa, em, cells)


def c3_batched_groups(n_cells: int = 2_097_152, D: int = 84, n_src: int = 10_000,
                      n_modes: int = 32, sigma: float = 2.0, tau: float = 10.0,
                      group_scale=(1.0, 0.3, 0.1, 0.03), n_pbc: int = 3) -> dict:
    """Clustered periodic mesh (seeds ~ lognormal density, sigma 2, 32^3 white modes),
    84 directions x 4 groups, 10,000 sources, 3 periodic-boundary passes.
    kappa proportional to the local density (kappa = n_H sigma_H) at mean optical depth 10."""
    r_pos, r_kap, r_src, _ = _streams(3)
    rho = lognormal_density_grid(n_modes, sigma, r_kap)
    pts = clustered_points(n_cells, rho, r_pos)
    mesh = voronoi_mesh(pts, periodic=True)
    C = len(mesh["cell_volume"])
    k0 = scale_to_mean_tau(density_at(mesh["points"], rho), mesh["cell_volume"], tau)
    kappa = k0[:, None] * np.asarray(group_scale)[None, :]
    cells, lum = point_sources(C, n_src, r_src)
    em = np.zeros((C, len(group_scale)))
    em[cells, :] = lum[:, None]
    return _workload("c3_batched_groups", [mesh], D, kappa, em, cells, boundary="periodic",
                     n_pbc=n_pbc)


def c4_differentiation(n_side: int = 64, D: int = 48, n_src: int = 50, tau: float = 10.0) -> dict:
    """c2's mesh recipe, 48 directions, 50 sources, lognormal kappa (sigma 1, mean 10)."""
    r_pos, r_kap, r_src, _ = _streams(4)
    mesh = jittered_lattice_mesh(n_side, r_pos)
    C = len(mesh["cell_volume"])
    kappa = lognormal_kappa(mesh["cell_volume"], r_kap, 1.0, tau)
    cells, lum = point_sources(C, n_src, r_src)
    em = np.zeros(C)
    em[cells] = lum
    return _workload("c4_differentiation", [mesh], D, kappa, em, cells)


def c5_uneven_scatter(n_meshes: int = 64, lo: int = 4096, hi: int = 262_144, D: int = 24,
                      n_src: int = 16, tau: float = 10.0, albedo: float = 0.5,
                      n_scat: int = 20) -> dict:
    """64 independent uniform-seed meshes, sizes log-uniform in [4096, 262144], vacuum,
    24 directions, lognormal kappa (mean 10) as extinction, albedo 0.5, 20 source iterations."""
    r_pos, r_kap, r_src, r_size = _streams(5)
    sizes = np.round(np.exp(r_size.uniform(np.log(lo), np.log(hi), size=n_meshes))).astype(int)
    meshes, kap, em, srcs = [], [], [], []
    off = 0
    for n in sizes:
        m = uniform_mesh(int(n), r_pos)
        C = len(m["cell_volume"])
        meshes.append(m)
        kap.append(lognormal_kappa(m["cell_volume"], r_kap, 1.0, tau))
        cells, lum = point_sources(C, n_src, r_src)
        e = np.zeros(C)
        e[cells] = lum
        em.append(e)
        srcs.append(cells + off)
        off += C
    return _workload("c5_uneven_scatter", meshes, D, np.concatenate(kap), np.concatenate(em),
                     np.concatenate(srcs), albedo=albedo, n_scat=n_scat)


def lattice_workload(n: int, dirs: np.ndarray, kappa: float, src_cells, lum, periodic=False,
                     G: int = 1) -> dict:
    """Cubic-lattice workload used by the closed-form checks."""
    mesh = lattice_mesh(n, periodic=periodic)
    C = n ** 3
    em = np.zeros((C, G))
    em[np.asarray(src_cells), :] = np.asarray(lum, dtype=np.float64).reshape(-1, 1)
    w = _workload("lattice", [mesh], 8, np.full((C, G), kappa), em, src_cells,
                  boundary="periodic" if periodic else "vacuum")
    w["dirs"] = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    return w


KPC_CM = 3.0856775814913673e21


def hii_rtype(n_side: int = 32, D: int = 84) -> dict:
    """R-type HII region (sec. 3.1.1): an n_side^3 lattice of a cube of side
    12.8 kpc, uniform neutral hydrogen n_H = 1e-3 cm^-3, one source of 1e49
    ionising photons/s in the central cell (emission in units of that rate),
    sigma_H = 5.38e-18 cm^2 and alpha_B = 2.59e-13 cm^3/s (tests section).
    kappa is the fully neutral extinction per mesh length unit; `hii` holds the
    parameters of the time stepping (step cap and end time in recombination
    times, the step-limit factor)."""
    c = n_side // 2
    hii = dict(n_H=1e-3, sigma_H=5.38e-18, alpha_B=2.59e-13, photon_rate=1e49,
               length_unit=12.8 * KPC_CM, dt_max_trec=0.05, t_end_trec=1.5, courant=1.0)
    w = lattice_workload(n_side, direction_set(D), hii["n_H"] * hii["sigma_H"] * hii["length_unit"],
                         [c + n_side * (c + n_side * c)], [1.0])
    w["name"] = "hii_rtype"
    w["law"] = "exp"
    w["hii"] = hii
    w["source_pos"] = np.full(3, (c + 0.5) / n_side)
    return w


def small_random(n_cells: int, D: int, G: int = 1, seed: int = 0, periodic: bool = False,
                 n_src: int = 3, tau: float = 3.0, sigma: float = 1.0, n_meshes: int = 1,
                 **opts) -> dict:
    """Small seeded random workload for tests (several meshes if n_meshes > 1)."""
    r_pos, r_kap, r_src, r_size = _streams(100, extra=seed + 1)
    meshes, kap, em, srcs = [], [], [], []
    off = 0
    for m_i in range(n_meshes):
        n = n_cells if m_i == 0 else int(r_size.integers(max(8, n_cells // 4), n_cells + 1))
        m = uniform_mesh(n, r_pos, periodic=periodic)
        C = len(m["cell_volume"])
        meshes.append(m)
        base = lognormal_kappa(m["cell_volume"], r_kap, sigma, tau)
        kap.append(base[:, None] * np.linspace(1.0, 0.2, G)[None, :])
        cells, lum = point_sources(C, n_src, r_src)
        e = np.zeros((C, G))
        e[cells, :] = lum[:, None]
        em.append(e)
        srcs.append(cells + off)
        off += C
    return _workload("small_random", meshes, D, np.concatenate(kap), np.concatenate(em),
                     np.concatenate(srcs), boundary="periodic" if periodic else "vacuum", **opts)


def many_faces(n_cells: int = 100, D: int = 24, G: int = 1, seed: int = 0, n_src: int = 4,
               tau: float = 2.0, **opts) -> dict:
    """Workload on the complete-graph test mesh (every cell has n_cells + 5 faces)."""
    from .mesh import complete_graph_mesh
    mesh = complete_graph_mesh(n_cells, seed)
    r_pos, r_kap, r_src, _ = _streams(101, extra=seed + 1)
    kap = lognormal_kappa(mesh["cell_volume"], r_kap, 1.0, tau)
    cells, lum = point_sources(n_cells, n_src, r_src)
    em = np.zeros((n_cells, G))
    em[cells, :] = lum[:, None]
    return _workload("many_faces", [mesh], D, kap[:, None] * np.linspace(1.0, 0.3, G)[None, :], em,
                     cells, **opts)


CONFIGS = {
    "c1": c1_plain_small,
    "c2": c2_plain_scale,
    "c3": c3_batched_groups,
    "c4": c4_differentiation,
    "c5": c5_uneven_scatter,
}
