"""ctypes binding of libsweep.so: the C ABI of include/sweep.h, same names, marshalling only.

There is no fallback: if the HIP library is missing or fails to load, every call
raises SweepLibraryError.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsweep.so")

SWEEP_OK = 0
STATUS_NAMES = {0: "SWEEP_OK", -1: "SWEEP_ERR_INVALID_ARG", -2: "SWEEP_ERR_CYCLE",
                -3: "SWEEP_ERR_OOM", -4: "SWEEP_ERR_HIP", -5: "SWEEP_ERR_NOT_BUILT",
                -6: "SWEEP_ERR_UNSUPPORTED"}
SWEEP_N_TOTALS = 8
SWEEP_BOUNDARY_VACUUM, SWEEP_BOUNDARY_PERIODIC = 0, 1
SWEEP_FORM_BATCHED, SWEEP_FORM_PLAIN = 0, 1
SWEEP_LAW_UPWIND, SWEEP_LAW_EXP = 0, 1
SWEEP_SCHEME_AREA, SWEEP_SCHEME_ALIGNED = 0, 1

EXPORTED = ("sweep_last_error", "sweep_build_dag", "sweep_destroy_dag", "sweep_dag_info",
            "sweep_dag_export", "sweep_saved_bytes", "sweep_forward", "sweep_adjoint",
            "sweep_tune", "sweep_ion_step", "sweep_profile_enable", "sweep_profile_reset",
            "sweep_profile_read", "sweep_sync", "sweep_dag_depths", "sweep_dag_level_widths",
            "sweep_ion_kappa", "sweep_ion_step_noalloc")


class SweepLibraryError(RuntimeError):
    """The native library is missing or could not be loaded."""


class SweepError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class sweep_mesh_t(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32), ("n_half_faces", ctypes.c_int64),
                ("face_ptr", ctypes.c_void_p), ("face_nbr", ctypes.c_void_p),
                ("face_twin", ctypes.c_void_p), ("face_shift", ctypes.c_void_p),
                ("face_area", ctypes.c_void_p), ("face_normal", ctypes.c_void_p),
                ("cell_volume", ctypes.c_void_p)]


class sweep_build_opts_t(ctypes.Structure):
    _fields_ = [("eps_tie", ctypes.c_double), ("validate", ctypes.c_int32),
                ("kahn_counters", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("n_aligned", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class sweep_dag_info_t(ctypes.Structure):
    _fields_ = [("n_meshes", ctypes.c_int32), ("n_dirs", ctypes.c_int32),
                ("n_cells", ctypes.c_int64), ("n_tasks", ctypes.c_int64),
                ("n_up_entries", ctypes.c_int64), ("n_down_entries", ctypes.c_int64),
                ("max_depth", ctypes.c_int32), ("min_depth", ctypes.c_int32),
                ("mean_depth", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("kahn_lds_counters", ctypes.c_int32), ("scheme", ctypes.c_int32)]


class sweep_ion_params_t(ctypes.Structure):
    _fields_ = [("n_H", ctypes.c_double), ("sigma_H", ctypes.c_double), ("alpha_B", ctypes.c_double),
                ("photon_rate", ctypes.c_double), ("length_unit", ctypes.c_double),
                ("dt_max", ctypes.c_double), ("courant", ctypes.c_double),
                ("reserved", ctypes.c_double * 5)]


class sweep_fwd_opts_t(ctypes.Structure):
    _fields_ = [("boundary", ctypes.c_int32), ("n_pbc", ctypes.c_int32),
                ("albedo", ctypes.c_double), ("n_scat", ctypes.c_int32),
                ("form", ctypes.c_int32), ("block", ctypes.c_int32), ("ring", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("law", ctypes.c_int32), ("merge", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("pbc_tol", ctypes.c_double),
                ("check", ctypes.c_int32), ("grid", ctypes.c_int32), ("pack", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsweep.so (raises SweepLibraryError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise SweepLibraryError("%s is not built; run `python -m paper_2207_12848_amd.build`" % path)
    try:
        lib = ctypes.CDLL(path)
    except OSError as e:  # pragma: no cover - depends on the machine
        raise SweepLibraryError("cannot load %s: %s" % (path, e)) from e
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "sweep_last_error": (ctypes.c_char_p, []),
        "sweep_build_dag": (ctypes.c_int, [P, I32, P, I32, P, P, P]),
        "sweep_destroy_dag": (ctypes.c_int, [P]),
        "sweep_dag_info": (ctypes.c_int, [P, P]),
        "sweep_dag_export": (ctypes.c_int, [P, P, P, P, P]),
        "sweep_saved_bytes": (SZ, [P, I32, P]),
        "sweep_forward": (ctypes.c_int, [P, I32, P, P, P, P, P, P, P, SZ, P]),
        "sweep_adjoint": (ctypes.c_int, [P, I32, P, P, P, P, SZ, P, P, P, P, P]),
        "sweep_tune": (ctypes.c_int, [P, I32, P, P, P, I32, P, P, P]),
        "sweep_ion_step": (ctypes.c_int, [P, P, P, ctypes.c_double, P, P, P, P]),
        "sweep_profile_enable": (ctypes.c_int, [I32]),
        "sweep_profile_reset": (ctypes.c_int, []),
        "sweep_profile_read": (ctypes.c_int, [ctypes.c_char_p, P, P]),
        "sweep_sync": (ctypes.c_int, [P, P]),
        "sweep_dag_depths": (ctypes.c_int, [P, P]),
        "sweep_dag_level_widths": (ctypes.c_int, [P, I32, P, I32, P]),
        "sweep_ion_kappa": (ctypes.c_int, [P, P, P, P, P]),
        "sweep_ion_step_noalloc": (ctypes.c_int, [P, P, P, ctypes.c_double, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != SWEEP_OK:
        raise SweepError(status, load().sweep_last_error().decode())


# Thin wrappers with the C names; pointers are ints (device addresses) or ctypes objects.
def sweep_last_error() -> str:
    return load().sweep_last_error().decode()


def sweep_build_dag(meshes, n_meshes, dirs, n_dirs, opts, stream, out) -> int:
    return load().sweep_build_dag(meshes, n_meshes, dirs, n_dirs, opts, stream, out)


def sweep_destroy_dag(dag) -> int:
    return load().sweep_destroy_dag(dag)


def sweep_dag_info(dag, info) -> int:
    return load().sweep_dag_info(dag, info)


def sweep_dag_export(dag, level, order, indeg, stream) -> int:
    return load().sweep_dag_export(dag, level, order, indeg, stream)


def sweep_saved_bytes(dag, G, opts) -> int:
    return load().sweep_saved_bytes(dag, G, opts)


def sweep_forward(dag, G, kappa, emission, opts, J, absorbed, totals, saved, saved_bytes,
                  stream) -> int:
    return load().sweep_forward(dag, G, kappa, emission, opts, J, absorbed, totals, saved,
                                saved_bytes, stream)


def sweep_adjoint(dag, G, kappa, emission, opts, saved, saved_bytes, dL_dJ, dL_dabsorbed,
                  dL_dkappa, dL_demission, stream) -> int:
    return load().sweep_adjoint(dag, G, kappa, emission, opts, saved, saved_bytes, dL_dJ,
                                dL_dabsorbed, dL_dkappa, dL_demission, stream)


def sweep_tune(dag, G, kappa, emission, opts, reps, best, best_ms, stream) -> int:
    return load().sweep_tune(dag, G, kappa, emission, opts, reps, best, best_ms, stream)


def sweep_ion_step(dag, absorbed, params, t_left, neutral, kappa, dt, stream) -> int:
    return load().sweep_ion_step(dag, absorbed, params, t_left, neutral, kappa, dt, stream)


def sweep_profile_enable(on: int) -> int:
    return load().sweep_profile_enable(on)


def sweep_profile_reset() -> int:
    return load().sweep_profile_reset()


def sweep_profile_read(kernel, launches, total_ms) -> int:
    return load().sweep_profile_read(kernel, launches, total_ms)


def sweep_sync(dag, stream) -> int:
    return load().sweep_sync(dag, stream)


def sweep_dag_depths(dag, depth) -> int:
    return load().sweep_dag_depths(dag, depth)


def sweep_dag_level_widths(dag, mesh, width, n_levels, stream) -> int:
    return load().sweep_dag_level_widths(dag, mesh, width, n_levels, stream)


def sweep_ion_kappa(dag, params, neutral, kappa, stream) -> int:
    return load().sweep_ion_kappa(dag, params, neutral, kappa, stream)


def sweep_ion_step_noalloc(dag, absorbed, params, t_left, neutral, kappa, dt, stream) -> int:
    return load().sweep_ion_step_noalloc(dag, absorbed, params, t_left, neutral, kappa, dt, stream)
