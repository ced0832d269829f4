"""MI355X transport sweep (Peter et al. 2022, "The Sweep Method for radiative Transfer in Arepo").

Python front-end of libsweep.so (include/sweep.h).  Every step of the sweep runs
in the library's HIP kernels; this module only moves arguments across the C ABI,
with torch providing device memory and the current stream.  There is no CPU
fallback: without the built library every call raises SweepLibraryError.

    dag = build_dag([mesh], dirs)                  # per-direction dependency graphs
    J, absorbed, totals = forward(dag, kappa, emission)
    J, absorbed = SweepFunction.apply(kappa, emission, dag, opts)   # differentiable
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _binding as B
from ._binding import (SweepError, SweepLibraryError, sweep_adjoint, sweep_build_dag,  # noqa: F401
                       sweep_dag_export, sweep_dag_info, sweep_destroy_dag, sweep_forward,
                       sweep_last_error, sweep_profile_enable, sweep_profile_read,
                       sweep_ion_step, sweep_profile_reset, sweep_saved_bytes, sweep_tune,
                       sweep_sync, sweep_dag_depths, sweep_dag_level_widths, sweep_ion_kappa,
                       sweep_ion_step_noalloc)

TOTAL_NAMES = ("emitted", "absorbed", "escaped", "pbc_in", "pbc_out", "scat_net", "pbc_err_max",
               "pbc_err_l1")

__all__ = ["Dag", "build_dag", "forward", "adjoint", "tune", "ion_step", "evolve_ionisation",
           "SweepFunction", "upload_mesh",
           "SweepError", "SweepLibraryError", "TOTAL_NAMES"] + list(B.EXPORTED)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def upload_mesh(mesh: dict, device="cuda") -> dict:
    """Copy a mesh (dict of numpy arrays, see synth.mesh) to device tensors."""
    def t(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)
    out = dict(face_ptr=t(mesh["face_ptr"], torch.int64), face_nbr=t(mesh["face_nbr"], torch.int32),
               face_twin=t(mesh["face_twin"], torch.int32) if "face_twin" in mesh else None,
               face_shift=t(mesh["face_shift"], torch.int8) if mesh.get("periodic") else None,
               face_area=t(mesh["face_area"], torch.float64),
               face_normal=t(np.asarray(mesh["face_normal"]).reshape(-1), torch.float64),
               cell_volume=t(mesh["cell_volume"], torch.float64))
    return out


def _fwd_opts(boundary="vacuum", n_pbc=1, albedo=0.0, n_scat=1, form="batched", block=0, ring=0,
              use_graph=False, law="upwind", merge=False, warm_start=False,
              pbc_tol=0.0, check=False, grid=0, pack=0) -> B.sweep_fwd_opts_t:
    o = B.sweep_fwd_opts_t()
    o.boundary = {"vacuum": B.SWEEP_BOUNDARY_VACUUM, "periodic": B.SWEEP_BOUNDARY_PERIODIC}[boundary]
    o.n_pbc = int(n_pbc)
    o.albedo = float(albedo)
    o.n_scat = int(n_scat)
    o.form = {"batched": B.SWEEP_FORM_BATCHED, "plain": B.SWEEP_FORM_PLAIN}[form]
    o.block = int(block)
    o.ring = int(ring)
    o.use_graph = int(bool(use_graph))
    o.law = {"upwind": B.SWEEP_LAW_UPWIND, "exp": B.SWEEP_LAW_EXP}[law]
    o.merge = int(bool(merge))
    o.warm_start = int(bool(warm_start))
    o.pbc_tol = float(pbc_tol)
    o.check = int(bool(check))
    o.grid = int(grid)
    o.pack = int(pack)
    return o


class Dag:
    """Owner of a sweep_dag_t handle."""

    def __init__(self, handle: ctypes.c_void_p, mesh_cells, n_dirs: int, device):
        self._h = handle
        self.mesh_cells = list(mesh_cells)
        self.n_cells = int(sum(mesh_cells))
        self.n_dirs = int(n_dirs)
        self.device = device

    @property
    def handle(self):
        if self._h is None:
            raise SweepError(-5, "DAG was destroyed")
        return self._h

    def info(self) -> dict:
        i = B.sweep_dag_info_t()
        B.check(sweep_dag_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in B.sweep_dag_info_t._fields_}

    def depths(self) -> np.ndarray:
        """Critical-path length of every (mesh, direction) graph, int32 [n_meshes, n_dirs]."""
        d = np.empty(len(self.mesh_cells) * self.n_dirs, np.int32)
        B.check(sweep_dag_depths(self.handle, d.ctypes.data))
        return d.reshape(len(self.mesh_cells), self.n_dirs)

    def level_widths(self, mesh: int = -1, stream=None) -> np.ndarray:
        """Tasks per level summed over the directions of `mesh` (-1: every mesh), int64."""
        n = int(self.info()["max_depth"])
        w = np.zeros(n, np.int64)
        B.check(sweep_dag_level_widths(self.handle, int(mesh), w.ctypes.data, n, _stream(stream)))
        return w

    def sync(self, stream=None) -> None:
        """Synchronise the stream; raises SweepError if earlier calls met invalid input."""
        B.check(sweep_sync(self.handle, _stream(stream)))

    def export(self, stream=None):
        """(level, order, indeg) as int32 numpy arrays laid out [mesh][direction][cell]."""
        T = self.n_cells * self.n_dirs
        lv = np.empty(T, np.int32)
        od = np.empty(T, np.int32)
        ind = np.empty(T, np.int32)
        B.check(sweep_dag_export(self.handle, lv.ctypes.data, od.ctypes.data, ind.ctypes.data,
                                 _stream(stream)))
        return lv, od, ind

    def split(self, arr):
        """Split an exported [T] array into per-mesh [D, C_m] views."""
        out, off = [], 0
        for C in self.mesh_cells:
            out.append(arr[off:off + self.n_dirs * C].reshape(self.n_dirs, C))
            off += self.n_dirs * C
        return out

    def saved_bytes(self, G: int, n_scat: int = 1, **opts) -> int:
        """Bytes of the `saved` workspace for these forward options."""
        return int(sweep_saved_bytes(self.handle, G, ctypes.byref(_fwd_opts(n_scat=n_scat, **opts))))

    def close(self):
        if self._h is not None:
            sweep_destroy_dag(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_dag(meshes, dirs, eps: float = 1e-12, validate: bool = True, device="cuda",
              stream=None, kahn_counters: str = "auto", scheme: str = "area",
              n_aligned: int = 3) -> Dag:
    """Build the dependency graphs of `meshes` (numpy dicts or upload_mesh() results).
    kahn_counters: "auto", "lds" or "global" (where the level computation counts).
    scheme: transport scheme "area" (a) or "aligned" (b, the outflow shared by the
    n_aligned most aligned outflow faces; needs face_twin)."""
    B.load()
    dev = [m if isinstance(m.get("face_ptr"), torch.Tensor) else upload_mesh(m, device)
           for m in meshes]
    arr = (B.sweep_mesh_t * len(dev))()
    for i, m in enumerate(dev):
        arr[i].n_cells = int(m["cell_volume"].numel())
        arr[i].n_half_faces = int(m["face_nbr"].numel())
        arr[i].face_ptr = _ptr(m["face_ptr"])
        arr[i].face_nbr = _ptr(m["face_nbr"])
        arr[i].face_twin = _ptr(m.get("face_twin"))
        arr[i].face_shift = _ptr(m.get("face_shift"))
        arr[i].face_area = _ptr(m["face_area"])
        arr[i].face_normal = _ptr(m["face_normal"])
        arr[i].cell_volume = _ptr(m["cell_volume"])
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    opts = B.sweep_build_opts_t()
    opts.eps_tie = float(eps)
    opts.validate = int(bool(validate))
    opts.kahn_counters = {"auto": 0, "lds": 1, "global": 2}[kahn_counters]
    opts.scheme = {"area": B.SWEEP_SCHEME_AREA, "aligned": B.SWEEP_SCHEME_ALIGNED}[scheme]
    opts.n_aligned = int(n_aligned)
    h = ctypes.c_void_p()
    B.check(sweep_build_dag(arr, len(dev), d.ctypes.data, len(d), ctypes.byref(opts),
                            _stream(stream), ctypes.byref(h)))
    return Dag(h, [int(m["cell_volume"].numel()) for m in dev], len(d), device)


def _check_field(t, C, G, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous() and t.numel() == C * G):
        raise ValueError("%s must be a contiguous float32 CUDA tensor with %d elements" % (name, C * G))


def forward(dag: Dag, kappa: torch.Tensor, emission: torch.Tensor, save_for_adjoint: bool = False,
            stream=None, saved: torch.Tensor = None, **opts):
    """Forward sweep.  kappa/emission: float32 CUDA [C_total, G].  Returns
    (J [C,G], absorbed [C,G], totals [n_meshes, G, 8] float64[, saved workspace]).
    `saved`: an existing workspace to fill (and, with warm_start=True, to take the
    first pass's periodic inflow from); it is returned as the fourth element."""
    C = dag.n_cells
    G = kappa.numel() // max(C, 1)
    _check_field(kappa, C, G, "kappa")
    _check_field(emission, C, G, "emission")
    o = _fwd_opts(**opts)
    J = torch.empty((C, G), dtype=torch.float32, device=kappa.device)
    A = torch.empty_like(J)
    tot = torch.empty((len(dag.mesh_cells), G, B.SWEEP_N_TOTALS), dtype=torch.float64,
                      device=kappa.device)
    nbytes = 0
    if saved is not None:
        nbytes = saved.numel() * saved.element_size()
        save_for_adjoint = True
    elif save_for_adjoint:
        nbytes = int(sweep_saved_bytes(dag.handle, G, ctypes.byref(o)))
        saved = torch.empty(nbytes // 4, dtype=torch.float32, device=kappa.device)
    B.check(sweep_forward(dag.handle, G, _ptr(kappa), _ptr(emission), ctypes.byref(o), _ptr(J),
                          _ptr(A), _ptr(tot), _ptr(saved), nbytes, _stream(stream)))
    if save_for_adjoint:
        return J, A, tot, saved
    return J, A, tot


def adjoint(dag: Dag, kappa, emission, saved, dL_dJ, dL_dabsorbed, stream=None, **opts):
    """Adjoint sweep: returns (dL/dkappa, dL/demission) as float32 CUDA [C_total, G]."""
    C = dag.n_cells
    G = kappa.numel() // max(C, 1)
    for t, n in ((kappa, "kappa"), (emission, "emission"), (dL_dJ, "dL_dJ"),
                 (dL_dabsorbed, "dL_dabsorbed")):
        _check_field(t, C, G, n)
    o = _fwd_opts(**opts)
    dk = torch.empty((C, G), dtype=torch.float32, device=kappa.device)
    de = torch.empty_like(dk)
    B.check(sweep_adjoint(dag.handle, G, _ptr(kappa), _ptr(emission), ctypes.byref(o), _ptr(saved),
                          saved.numel() * saved.element_size(), _ptr(dL_dJ), _ptr(dL_dabsorbed),
                          _ptr(dk), _ptr(de), _stream(stream)))
    return dk, de


def tune(dag: Dag, kappa: torch.Tensor, emission: torch.Tensor, reps: int = 3, stream=None,
         **opts) -> dict:
    """Autotune the sweep's launch shape on this DAG: returns {"block", "ring", "ms"}
    (pass block= and ring= to forward/adjoint)."""
    C = dag.n_cells
    G = kappa.numel() // max(C, 1)
    _check_field(kappa, C, G, "kappa")
    _check_field(emission, C, G, "emission")
    o = _fwd_opts(**opts)
    best = B.sweep_fwd_opts_t()
    ms = ctypes.c_double()
    B.check(sweep_tune(dag.handle, G, _ptr(kappa), _ptr(emission), ctypes.byref(o), int(reps),
                       ctypes.byref(best), ctypes.byref(ms), _stream(stream)))
    return {"block": int(best.block), "ring": int(best.ring), "pack": int(best.pack), "ms": float(ms.value)}


def ion_step(dag: Dag, absorbed: torch.Tensor, neutral: torch.Tensor, kappa: torch.Tensor,
             params: dict, t_left: float, stream=None, no_alloc: bool = False) -> float:
    """One photoionisation chemistry step (sweep_ion_step): updates `neutral` (float64
    CUDA [C]) and writes `kappa` (float32 CUDA [C, 1]) in place; returns the step (s).
    params: n_H, sigma_H, alpha_B, photon_rate, length_unit, dt_max (s), courant.
    no_alloc: use sweep_ion_step_noalloc (the library's static scratch word; calls
    that overlap on one GPU race)."""
    C = dag.n_cells
    if not (neutral.is_cuda and neutral.dtype == torch.float64 and neutral.numel() == C
            and neutral.is_contiguous()):
        raise ValueError("neutral must be a contiguous float64 CUDA tensor with %d elements" % C)
    _check_field(absorbed, C, 1, "absorbed")
    _check_field(kappa, C, 1, "kappa")
    p = B.sweep_ion_params_t()
    for k in ("n_H", "sigma_H", "alpha_B", "photon_rate", "length_unit", "dt_max", "courant"):
        setattr(p, k, float(params[k]))
    dt = ctypes.c_double()
    fn = sweep_ion_step_noalloc if no_alloc else sweep_ion_step
    B.check(fn(dag.handle, _ptr(absorbed), ctypes.byref(p), float(t_left), _ptr(neutral), _ptr(kappa),
               ctypes.byref(dt), _stream(stream)))
    return float(dt.value)


def evolve_ionisation(dag: Dag, emission: torch.Tensor, params: dict, t_end: float,
                      neutral: torch.Tensor = None, record=None, max_steps: int = 10_000_000,
                      **opts):
    """Time-step a photoionisation run (sweep under the exponential law, then
    ion_step) from `neutral` (default: fully neutral) until t_end seconds.
    Returns (t, neutral, steps); calls record(step, t, neutral, absorbed, dt) after
    every step when given.  `dag` may be a list of DAGs of the same meshes built for
    rotated direction sets: step k sweeps dag[(k0 + k) % len(dag)], k0 = opts
    "step0" (default 0)."""
    dags = list(dag) if isinstance(dag, (list, tuple)) else [dag]
    step0 = int(opts.pop("step0", 0))
    dag = dags[0]
    C = dag.n_cells
    dev = emission.device
    y = torch.ones(C, dtype=torch.float64, device=dev) if neutral is None else neutral
    kappa = torch.empty((C, 1), dtype=torch.float32, device=dev)
    p = B.sweep_ion_params_t()
    for k in ("n_H", "sigma_H", "length_unit"):
        setattr(p, k, float(params[k]))
    B.check(sweep_ion_kappa(dag.handle, ctypes.byref(p), _ptr(y), _ptr(kappa), _stream(None)))
    o = dict(opts, law="exp")
    t, step = 0.0, 0
    while t < t_end and step < max_steps:
        dg = dags[(step0 + step) % len(dags)]
        _, A, _ = forward(dg, kappa, emission, **o)
        dt = ion_step(dg, A, y, kappa, params, t_end - t)
        t += dt
        step += 1
        if record is not None:
            record(step - 1, t, y, A, dt)
    return t, y, step


KERNELS = ("count", "kahn", "fill", "prep", "sweep_fwd", "sweep_adj", "reduce")


def profile_enable(on: bool = True) -> None:
    """Bracket the library's kernels with HIP events (see kernel_times)."""
    B.check(sweep_profile_enable(int(bool(on))))


def profile_reset() -> None:
    B.check(sweep_profile_reset())


def kernel_times() -> dict:
    """{kernel: (launches, total ms)} recorded since the last profile_reset()."""
    out = {}
    for k in KERNELS:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        B.check(sweep_profile_read(k.encode(), ctypes.byref(n), ctypes.byref(ms)))
        out[k] = (int(n.value), float(ms.value))
    return out


class SweepFunction(torch.autograd.Function):
    """(kappa, emission) -> (J, absorbed), differentiable through the hand-written adjoint."""

    @staticmethod
    def forward(ctx, kappa, emission, dag, opts=None):
        opts = dict(opts or {})
        J, A, tot, saved = forward(dag, kappa.contiguous(), emission.contiguous(),
                                   save_for_adjoint=True, **opts)
        ctx.dag, ctx.opts = dag, opts
        ctx.save_for_backward(kappa, emission, saved)
        ctx.mark_non_differentiable(tot)
        return J, A, tot

    @staticmethod
    def backward(ctx, gJ, gA, gtot):
        kappa, emission, saved = ctx.saved_tensors
        gJ = torch.zeros_like(kappa) if gJ is None else gJ.contiguous().float()
        gA = torch.zeros_like(kappa) if gA is None else gA.contiguous().float()
        dk, de = adjoint(ctx.dag, kappa.contiguous(), emission.contiguous(), saved, gJ, gA,
                         **ctx.opts)
        return dk, de, None, None
