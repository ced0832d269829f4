"""Dense direct solves of the discretised transport equations (test helper).

Independent of the oracle's sweep: the per-direction system is assembled as a
matrix straight from the face list and solved with numpy.linalg.solve, with no
dependency graph, ordering or queue.  For direction Omega (sec. 2.5/2.6):

    (Aperp_c + kappa_c V_c) phi_c - sum_{inflow faces f of c} A_f |n_f . Omega| phi_nbr(f) = S_c

With the exponential cell law (transmission e^{-tau} over the mean chord
V/Aperp, tau = kappa V / Aperp, capped at 40) the unknown is the exit flux
density x and the diagonal becomes Aperp e^{tau}; the cell average is r x with
r = Aperp (e^{tau} - 1) / (kappa V) (1 at kappa = 0).

Transport scheme (b) of sec. 2.6 (scheme="aligned"): a cell's outflow Aperp phi
is shared equally by its n outflow faces with the largest Omega . n (ties: the
lower face index), so the coupling is assembled from the sending side:
M[i, c] -= Aperp_c / n for every such face of c towards i.

cyclic=True also couples the periodic faces, giving the fixed point of the
periodic-boundary passes (sec. 2.7).  `dense_scatter_system` couples all
directions through the isotropic scattering term of eq. radiativeTransfer, giving
the fixed point of source iteration (algorithm 1).
"""
from __future__ import annotations

import numpy as np

EPS = 1e-12


def _faces(mesh):
    fp = mesh["face_ptr"]
    owner = np.repeat(np.arange(len(fp) - 1), np.diff(fp))
    periodic = bool(mesh.get("periodic"))
    shift = mesh["face_shift"] if periodic else np.zeros(len(owner), np.int8)
    return owner, mesh["face_nbr"], shift, mesh["face_area"], mesh["face_normal"]


TAU_CAP = 40.0


def _orient(normal, omega):
    """Omega . n per face, as (ox nx + oy ny) + oz nz in FP64 (elementwise, no FMA)."""
    o = np.asarray(omega, np.float64)
    return (normal[:, 0] * o[0] + normal[:, 1] * o[1]) + normal[:, 2] * o[2]


def aligned_choice(mesh, omega, eps=EPS, n_aligned=3):
    """Scheme (b): per face, the weight with which its owner's intensity leaves
    through it (Aperp / n on the owner's n most aligned outflow faces, else 0),
    and whether it carries radiation."""
    owner, nbr, shift, area, normal = _faces(mesh)
    C = len(mesh["cell_volume"])
    s = _orient(normal, omega)
    out = s > eps
    aperp = np.bincount(owner[out], weights=(area * np.abs(s))[out], minlength=C)
    fp = mesh["face_ptr"]
    wb = np.zeros(len(s))
    chosen = np.zeros(len(s), bool)
    for c in range(C):
        fs = [f for f in range(fp[c], fp[c + 1]) if out[f]]
        fs.sort(key=lambda f: (-s[f], f))
        n = min(n_aligned, len(fs))
        for f in fs[:n]:
            chosen[f] = True
            wb[f] = aperp[c] / n
    return wb, chosen


def direction_matrix(mesh, omega, kappa, cyclic=False, eps=EPS, law="upwind", scheme="area"):
    """M (C x C), the outflow weights of walls / periodic faces for one direction and
    r, the factor from the unknown to the cell average."""
    owner, nbr, shift, area, normal = _faces(mesh)
    C = len(mesh["cell_volume"])
    s = _orient(normal, omega) if scheme == "aligned" else normal @ np.asarray(omega, np.float64)
    w = area * np.abs(s)
    out = s > eps
    inn = s < -eps
    aperp = np.bincount(owner[out], weights=w[out], minlength=C)
    kV = kappa * mesh["cell_volume"]
    if law == "exp":
        tau = np.minimum(kV / aperp, TAU_CAP)
        M = np.diag(aperp * np.exp(tau))
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(kV > 0, aperp * np.expm1(tau) / kV, 1.0)
    else:
        M = np.diag(aperp + kV)
        r = np.ones(C)
    interior = nbr >= 0
    per = shift != 0
    if scheme == "aligned":
        wb, ch = aligned_choice(mesh, omega, eps)
        use = ch & interior & ((~per) | cyclic)
        np.add.at(M, (nbr[use], owner[use]), -wb[use])
        wall_out = np.bincount(owner[ch & ~interior], weights=wb[ch & ~interior], minlength=C)
        per_out = np.bincount(owner[ch & interior & per], weights=wb[ch & interior & per],
                              minlength=C)
        return M, wall_out, per_out, r
    use = inn & interior & ((~per) | cyclic)
    np.add.at(M, (owner[use], nbr[use]), -w[use])
    wall_out = np.bincount(owner[out & ~interior], weights=w[out & ~interior], minlength=C)
    per_out = np.bincount(owner[out & interior & per], weights=w[out & interior & per], minlength=C)
    return M, wall_out, per_out, r


def dense_forward(w, cyclic=False):
    """phi [D,C,G] per mesh, J, absorbed and (emitted, absorbed, escaped) per mesh/group."""
    dirs = w["dirs"]
    G = w["G"]
    kap = np.asarray(w["kappa"], np.float64)
    em = np.asarray(w["emission"], np.float64)
    D = len(dirs)
    law = w.get("law", "upwind")
    scheme = w.get("scheme", "area")
    off = 0
    Js, As, tots, phis = [], [], [], []
    for mesh in w["meshes"]:
        C = len(mesh["cell_volume"])
        k = kap[off:off + C]
        e = em[off:off + C]
        phi = np.zeros((D, C, G))
        avg = np.zeros((D, C, G))
        esc = np.zeros(G)
        for d in range(D):
            for g in range(G):
                M, wall, _, r = direction_matrix(mesh, dirs[d], k[:, g], cyclic, law=law,
                                                 scheme=scheme)
                phi[d, :, g] = np.linalg.solve(M, e[:, g] / D)
                avg[d, :, g] = r * phi[d, :, g]
                esc[g] += wall @ phi[d, :, g]
        js = avg.sum(axis=0)
        J = js / (4 * np.pi)
        A = k * mesh["cell_volume"][:, None] * js
        Js.append(J)
        As.append(A)
        tots.append(np.stack([e.sum(axis=0), A.sum(axis=0), esc], axis=1))
        phis.append(phi)
        off += C
    return dict(J=np.concatenate(Js), absorbed=np.concatenate(As), totals=np.stack(tots), phi=phis)


def dense_scatter_system(w, cyclic=False):
    """Fixed point of source iteration: all D directions solved together for one mesh, one group.

    Unknowns x[d,c]; equations M_d x_d - (a kappa V / D) sum_d' r_d' x_d' = L / D; returns
    the cell averages r_d x_d.  cyclic=True couples the periodic faces as well (the
    fixed point of periodic passes and source iteration together)."""
    (mesh,) = w["meshes"]
    dirs = w["dirs"]
    D = len(dirs)
    C = len(mesh["cell_volume"])
    k = np.asarray(w["kappa"], np.float64)[:, 0]
    L = np.asarray(w["emission"], np.float64)[:, 0]
    a = w["albedo"]
    V = mesh["cell_volume"]
    law = w.get("law", "upwind")
    big = np.zeros((D * C, D * C))
    rs = []
    for d in range(D):
        M, _, _, r = direction_matrix(mesh, dirs[d], k, cyclic=cyclic, law=law)
        rs.append(r)
        big[d * C:(d + 1) * C, d * C:(d + 1) * C] += M
    for d in range(D):
        for d2 in range(D):
            big[d * C:(d + 1) * C, d2 * C:(d2 + 1) * C] -= np.diag(a * k * V / D * rs[d2])
    x = np.linalg.solve(big, np.tile(L / D, D)).reshape(D, C)
    return x * np.stack(rs)


def dense_adjoint(w, gJ, gA, cyclic=False):
    """Gradients of L(J, absorbed), no scattering, upwind law: explicit matrices (cyclic:
    the periodic faces coupled, the fixed point of the periodic passes)."""
    dirs = w["dirs"]
    G = w["G"]
    kap = np.asarray(w["kappa"], np.float64)
    em = np.asarray(w["emission"], np.float64)
    D = len(dirs)
    scheme = w.get("scheme", "area")
    off = 0
    dk_all, de_all = [], []
    for mesh in w["meshes"]:
        C = len(mesh["cell_volume"])
        V = mesh["cell_volume"]
        dk = np.zeros((C, G))
        de = np.zeros((C, G))
        for g in range(G):
            k = kap[off:off + C, g]
            e = em[off:off + C, g]
            gj = gJ[off:off + C, g]
            ga = gA[off:off + C, g]
            gphi = gj / (4 * np.pi) + ga * k * V
            jsum = np.zeros(C)
            for d in range(D):
                M, _, _, _ = direction_matrix(mesh, dirs[d], k, cyclic=cyclic, scheme=scheme)
                phi = np.linalg.solve(M, e / D)
                lam = np.linalg.solve(M.T, gphi)
                jsum += phi
                de[:, g] += lam / D
                dk[:, g] -= V * lam * phi
            dk[:, g] += ga * V * jsum
        dk_all.append(dk)
        de_all.append(de)
        off += C
    return np.concatenate(dk_all), np.concatenate(de_all)


def brute_levels(mesh, omega, eps=EPS, scheme="area"):
    """Longest-path levels by repeated relaxation over the edge list (no queue)."""
    owner, nbr, shift, area, normal = _faces(mesh)
    C = len(mesh["cell_volume"])
    s = normal @ np.asarray(omega, np.float64)
    e = (s > eps) & (nbr >= 0) & (shift == 0)
    if scheme == "aligned":
        e = aligned_choice(mesh, omega, eps)[1] & (nbr >= 0) & (shift == 0)
    src, dst = owner[e], nbr[e]
    level = np.zeros(C, np.int64)
    for _ in range(C + 1):
        new = level.copy()
        np.maximum.at(new, dst, level[src] + 1)
        if np.array_equal(new, level):
            return level, src, dst
        level = new
    raise RuntimeError("cyclic")
