"""FP64 CPU oracle of the transport sweep -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2207_12848_amd``) and never imports it; both consume the seeded inputs
of ``synth``.

What is computed is documented in ``sweep_oracle.c`` (orientation of appendix A
and sec. 2.5, algorithm 2's FIFO schedule, transport schemes (a) and (b) of
sec. 2.6 (w["scheme"] = "area" or "aligned", w["n_aligned"] = 3) with a
first-order upwind cell balance or an exponential (e^{-tau}) cell law,
periodic passes of sec. 2.7, source
iteration of algorithm 1, and the adjoint).  This module only marshals numpy
arrays; every function loops over the independent meshes of a workload.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sweep_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

EPS_TIE = 1e-12
N_TOTALS = 8
TOTAL_NAMES = ("emitted", "absorbed", "escaped", "pbc_in", "pbc_out", "scat_net", "pbc_err_max",
               "pbc_err_l1")


class OracleError(RuntimeError):
    pass


class _Mesh(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32), ("face_ptr", ctypes.c_void_p),
                ("face_nbr", ctypes.c_void_p), ("face_shift", ctypes.c_void_p),
                ("face_area", ctypes.c_void_p), ("face_normal", ctypes.c_void_p),
                ("cell_volume", ctypes.c_void_p), ("face_twin", ctypes.c_void_p),
                ("scheme", ctypes.c_int32), ("n_aligned", ctypes.c_int32)]


SCHEMES = {"area": 0, "aligned": 1}


def build(force: bool = False) -> str:
    """Compile the oracle (gcc, FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_build_dag.restype = ctypes.c_int
        lib.orc_build_dag.argtypes = [P, ctypes.c_int32, P, ctypes.c_double, P, P, P, P]
        lib.orc_forward.restype = ctypes.c_int
        lib.orc_forward.argtypes = [P, ctypes.c_int32, P, ctypes.c_double, ctypes.c_int32, P, P,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, P, ctypes.c_double, P, P, P, P, P,
                                    P]
        lib.orc_adjoint.restype = ctypes.c_int
        lib.orc_adjoint.argtypes = [P, ctypes.c_int32, P, ctypes.c_double, ctypes.c_int32, P, P,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, P, ctypes.c_double, P, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _mesh_struct(mesh, scheme="area", n_aligned=3):
    """The C view of a mesh; scheme "area" (transport scheme (a)) or "aligned"
    (scheme (b): the outflow shared by the n_aligned most aligned faces)."""
    if scheme not in SCHEMES:
        raise OracleError("unknown transport scheme %r" % (scheme,))
    if scheme == "aligned" and mesh.get("face_twin") is None:
        raise OracleError("the aligned scheme needs the meshes' face_twin")
    keep = dict(face_ptr=_c(mesh["face_ptr"], np.int64), face_nbr=_c(mesh["face_nbr"], np.int32),
                face_shift=_c(mesh["face_shift"], np.int8) if mesh.get("periodic") else None,
                face_area=_c(mesh["face_area"], np.float64),
                face_normal=_c(mesh["face_normal"], np.float64),
                cell_volume=_c(mesh["cell_volume"], np.float64),
                face_twin=_c(mesh["face_twin"], np.int32) if mesh.get("face_twin") is not None
                else None)
    s = _Mesh(len(keep["cell_volume"]), _p(keep["face_ptr"]), _p(keep["face_nbr"]),
              _p(keep["face_shift"]), _p(keep["face_area"]), _p(keep["face_normal"]),
              _p(keep["cell_volume"]), _p(keep["face_twin"]), SCHEMES[scheme], int(n_aligned))
    return s, keep


def _scheme(w):
    return w.get("scheme", "area"), int(w.get("n_aligned", 3))


def _check(st, what):
    if st != 0:
        names = {-1: "invalid argument", -2: "cyclic dependency graph", -3: "out of memory",
                 -6: "unsupported"}
        raise OracleError("%s: %s (%d)" % (what, names.get(st, "error"), st))


LAWS = {"upwind": 0, "exp": 1}


def _law(w):
    law = w.get("law", "upwind")
    if law not in LAWS:
        raise OracleError("unknown cell law %r" % (law,))
    return LAWS[law]


def _offsets(meshes):
    off = [0]
    for m in meshes:
        off.append(off[-1] + len(m["cell_volume"]))
    return off


def build_dag(mesh: dict, dirs: np.ndarray, eps: float = EPS_TIE, scheme: str = "area",
              n_aligned: int = 3):
    """Levels, canonical order and upwind counts of every task of one mesh.

    Returns level [D,C], order [D,C] (cells of each direction sorted by (level, cell)),
    indeg [D,C] and depth [D]."""
    lib = _load()
    s, keep = _mesh_struct(mesh, scheme, n_aligned)
    dirs = _c(dirs, np.float64)
    D, C = len(dirs), s.n_cells
    level = np.zeros((D, C), np.int32)
    order = np.zeros((D, C), np.int32)
    indeg = np.zeros((D, C), np.int32)
    depth = np.zeros(D, np.int32)
    _check(lib.orc_build_dag(ctypes.byref(s), D, _p(dirs), eps, _p(level), _p(order), _p(indeg),
                             _p(depth)), "build_dag")
    return level, order, indeg, depth


def forward(w: dict, want_phi: bool = False, want_order: bool = False, eps: float = EPS_TIE,
            phi_init=None):
    """Sweep workload `w` (see synth.workloads; w["law"] is "upwind" (default) or "exp").
    Returns dict with J [C,G], absorbed [C,G], totals [n_meshes,G,8] and, on request, phi
    (list of [D,C,G] per mesh: the exit flux density), jsum_ckpt (list of [n_scat,C,G]) and
    the FIFO order (list of [D,C]).  w["merge"]: periodic passes and source iterations
    advance together (max(n_pbc, n_scat) passes).  w["pbc_tol"]: stop the periodic passes
    of an iteration once E < pbc_tol everywhere (n_pbc is then the maximum).
    phi_init: list of [D,C,G] exit flux
    densities per mesh whose periodic outflow feeds the first pass (warm start)."""
    lib = _load()
    dirs = _c(w["dirs"], np.float64)
    D, G = len(dirs), int(w["G"])
    kap = np.asarray(w["kappa"], np.float64).reshape(-1, G)
    em = np.asarray(w["emission"], np.float64).reshape(-1, G)
    off = _offsets(w["meshes"])
    periodic = w.get("boundary", "vacuum") == "periodic"
    n_pbc, albedo, n_scat = int(w.get("n_pbc", 1)), float(w.get("albedo", 0.0)), int(w.get("n_scat", 1))
    law = _law(w)
    merged = int(bool(w.get("merge", False)))
    J = np.zeros((off[-1], G))
    Ab = np.zeros((off[-1], G))
    totals = np.zeros((len(w["meshes"]), G, N_TOTALS))
    phis, ckpts, orders = [], [], []
    for mi, mesh in enumerate(w["meshes"]):
        s, keep = _mesh_struct(mesh, *_scheme(w))
        C = s.n_cells
        sl = slice(off[mi], off[mi + 1])
        k = _c(kap[sl], np.float64)
        e = _c(em[sl], np.float64)
        j = np.zeros((C, G))
        a = np.zeros((C, G))
        t = np.zeros((G, N_TOTALS))
        phi = np.zeros((D, C, G)) if want_phi else None
        ck = np.zeros((n_scat, C, G)) if want_phi else None
        qo = np.zeros((D, C), np.int32) if want_order else None
        pin = None if phi_init is None else _c(phi_init[mi], np.float64)
        _check(lib.orc_forward(ctypes.byref(s), D, _p(dirs), eps, G, _p(k), _p(e), int(periodic),
                               n_pbc, albedo, n_scat, law, merged, _p(pin),
                               float(w.get("pbc_tol", 0.0)), _p(j), _p(a), _p(t),
                               _p(phi), _p(ck), _p(qo)),
               "forward")
        J[sl], Ab[sl], totals[mi] = j, a, t
        phis.append(phi)
        ckpts.append(ck)
        orders.append(qo)
    out = dict(J=J, absorbed=Ab, totals=totals)
    if want_phi:
        out["phi"], out["jsum_ckpt"] = phis, ckpts
    if want_order:
        out["order"] = orders
    return out


def adjoint(w: dict, gJ: np.ndarray, gA: np.ndarray, eps: float = EPS_TIE, phi_init=None):
    """Gradients (dL/dkappa [C,G], dL/demission [C,G]) of a loss with dL/dJ = gJ and
    dL/dabsorbed = gA, through all source iterations and periodic passes (nested order,
    or the merged order when w["merge"]; with w["pbc_tol"], each iteration's passes
    up to where the forward's stopping test ends them, the count held fixed).
    phi_init: the warm start of forward() (held fixed)."""
    lib = _load()
    dirs = _c(w["dirs"], np.float64)
    D, G = len(dirs), int(w["G"])
    kap = np.asarray(w["kappa"], np.float64).reshape(-1, G)
    em = np.asarray(w["emission"], np.float64).reshape(-1, G)
    gJ = np.asarray(gJ, np.float64).reshape(-1, G)
    gA = np.asarray(gA, np.float64).reshape(-1, G)
    off = _offsets(w["meshes"])
    periodic = w.get("boundary", "vacuum") == "periodic"
    albedo, n_scat = float(w.get("albedo", 0.0)), int(w.get("n_scat", 1))
    law = _law(w)
    dk = np.zeros((off[-1], G))
    de = np.zeros((off[-1], G))
    for mi, mesh in enumerate(w["meshes"]):
        s, keep = _mesh_struct(mesh, *_scheme(w))
        C = s.n_cells
        sl = slice(off[mi], off[mi + 1])
        a = np.zeros((C, G))
        b = np.zeros((C, G))
        pin = None if phi_init is None else _c(phi_init[mi], np.float64)
        _check(lib.orc_adjoint(ctypes.byref(s), D, _p(dirs), eps, G, _p(_c(kap[sl], np.float64)),
                               _p(_c(em[sl], np.float64)), int(periodic),
                               int(w.get("n_pbc", 1)) if periodic else 1, albedo, n_scat, law,
                               int(bool(w.get("merge", False))), _p(pin),
                               float(w.get("pbc_tol", 0.0)),
                               _p(_c(gJ[sl], np.float64)), _p(_c(gA[sl], np.float64)), _p(a), _p(b)),
               "adjoint")
        dk[sl], de[sl] = a, b
    return dk, de


def num_threads() -> int:
    """OpenMP threads the oracle's direction loops run on."""
    lib = _load()
    lib.orc_num_threads.restype = ctypes.c_int
    return int(lib.orc_num_threads())


def set_threads(n: int) -> None:
    """Run the oracle's direction loops on n OpenMP threads."""
    lib = _load()
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads(int(n))


def absorbed_loss_grads(w: dict):
    """Upstream gradients of L = sum_c V_c kappa_a,c J_c = sum_c absorbed_c / (4 pi)."""
    G = int(w["G"])
    n = sum(len(m["cell_volume"]) for m in w["meshes"])
    return np.zeros((n, G)), np.full((n, G), 1.0 / (4.0 * np.pi))
