#!/usr/bin/env python3
"""Throughput of the MI355X transport sweep on one GPU.

One step is one pass of the whole hot path over one synthetic workload, every
input already resident in HBM:

    build_dag       orientation, counts and upwind/downwind lists (sec. 2.5, appendix A),
                    Kahn levels and the level schedule (algorithm 2's counters)
    forward         upwind cell balances in level order over every (mesh, direction),
                    groups packed per task, periodic passes (sec. 2.7) and source
                    iterations (algorithm 1) as the workload asks, J / absorbed rate and
                    FP64 totals
    adjoint         reverse sweep over the transposed graphs for the loss
                    L = sum_c absorbed_c / 4pi, giving dL/dkappa and dL/demission

value = cell-direction updates per second = (forward + adjoint updates per step) / time,
with C * D * G updates per pass.  The JSON line also carries the roofline of the
dominant kernel (HIP-event timing inside the timed region), the plain per-direction
form of the same step, and the FP64 CPU oracle timed on the host with its parity
check of the GPU outputs.

    python bench.py [--steps K] [--warmup W] [--workload c3_batched_groups]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
WORKLOADS = ("c1_plain_small", "c2_plain_scale", "c3_batched_groups", "c4_differentiation",
             "c5_uneven_scatter", "hii_rtype")
# kernels whose counters a PMC summary under profiles/ may cover, and their source
KERNEL_SOURCE = {"count": "dag.hip", "kahn": "dag.hip", "fill": "dag.hip", "prep": "sweep.hip",
                 "sweep_fwd": "sweep.hip", "sweep_adj": "sweep.hip", "reduce": "sweep.hip"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(kernel: str) -> str:
    p = os.path.join(HERE, "paper_2207_12848_amd", "csrc", KERNEL_SOURCE[kernel])
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# ------------------------------------------------------------------ byte model
def byte_model(kernel: str, s: dict) -> float:
    """Algorithmic HBM bytes of ONE launch of `kernel` (what the algorithm must move,
    FP32 fields, int32 ids; not what the implementation happens to move).

    s: C cells, H half-faces, T tasks (C * D), Eu upwind and Ed downwind entries
    (graph edges), G groups, launches per call."""
    C, H, T, Eu, Ed, G = s["C"], s["H"], s["T"], s["Eu"], s["Ed"], s["G"]
    face = 8 + 4 + 1 + 24.0  # area f64, neighbour i32, image code i8, normal 3 x f64
    if kernel == "count":
        # faces once; per task indeg, two row lengths, Aperp, boundary pair; downwind ids
        return H * face + C * 8 + T * 24 + Ed * 4
    if kernel == "kahn":
        # indeg and downwind ids in; schedule and its inverse out
        return T * 4 + Ed * 4 + T * 8
    if kernel == "fill":
        # faces once, own schedule position, neighbour positions; (id, w) entries out
        return H * face + C * 8 + T * 4 + (Eu + Ed) * (4 + 8)
    if kernel == "prep":
        # kappa, emission, V, Aperp in; denominator and source out (per task and group)
        return T * 4 + C * 4 + 2 * C * G * 4 + T * G * 8
    if kernel == "sweep_fwd":
        # task record (cell, row) + upwind (id, w) + per group: upwind phi gathers,
        # denominator, source, phi out
        return T * 8 + Eu * 8 + G * (Eu * 4 + T * 12)
    if kernel == "sweep_adj":
        return T * 8 + Ed * 8 + G * (Ed * 4 + T * 12)
    if kernel == "reduce":
        # phi of every direction in; J and absorbed out
        return T * G * 4 + 2 * C * G * 4
    raise KeyError(kernel)


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading)
    from the committed PMC summary profiles/pmc_<workload>.txt, or None when there is
    none or the kernel's source has changed since the counters were taken."""
    p = os.path.join(HERE, "profiles", "pmc_%s.txt" % workload)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        for line in f:
            tok = line.split()
            if line.startswith("#") or len(tok) != 5 or tok[0] != kernel:
                continue
            if tok[1] != source_digest(kernel):
                return None
            return float(tok[4])
    return None


# ------------------------------------------------------------------ workload
def make_workload(name: str) -> dict:
    from synth import workloads as W
    return getattr(W, name)()


def fwd_opts(w: dict, form: str = "batched", block: int = 0, ring: int = 0, pack: int = 0) -> dict:
    return dict(boundary=w.get("boundary", "vacuum"), n_pbc=int(w.get("n_pbc", 1)),
                albedo=float(w.get("albedo", 0.0)), n_scat=int(w.get("n_scat", 1)), form=form,
                block=block, ring=ring, pack=pack, law=w.get("law", "upwind"))


def updates_per_pass(w: dict) -> int:
    C = sum(len(m["cell_volume"]) for m in w["meshes"])
    return C * len(w["dirs"]) * int(w["G"])


# ------------------------------------------------------------------ CPU baseline
CPU_SAMPLE_UPDATES = 3.0e8  # about 10-30 s of the oracle on a few dozen host threads
PLAIN_SAMPLE_UPDATES = 1.5e8  # a few seconds of the plain form


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def sample_dirs(w: dict, n_updates: int, budget: float = CPU_SAMPLE_UPDATES) -> int:
    """Directions of the oracle's bounded sample (all of them when the step is small)."""
    D = len(w["dirs"])
    if n_updates <= budget:
        return D
    return max(1, int(D * budget / n_updates))


def parity(gpu: dict, ref: dict, dk, de) -> dict:
    """Element-wise comparison of GPU outputs with the oracle's (the bars of the tests)."""
    import numpy as np

    def rel(a, b, floor=1e-20):
        a = np.asarray(a, np.float64)
        b = np.asarray(b, np.float64)
        mask = np.abs(b) >= floor * np.abs(b).max()
        return dict(max_rel=float((np.abs(a - b)[mask] / np.abs(b)[mask]).max()),
                    l1_rel=float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300)))

    par = dict(J=rel(gpu["J"], ref["J"]), absorbed=rel(gpu["absorbed"], ref["absorbed"]))
    tg = np.asarray(gpu["totals"], np.float64)
    tr = ref["totals"]
    keep = np.abs(tr[..., :5]) > 0
    par["totals_max_rel"] = float(np.max(np.where(keep, np.abs(tg[..., :5] - tr[..., :5]) /
                                                  np.maximum(np.abs(tr[..., :5]), 1e-300), 0.0)))
    for key, a, b in (("dL_dkappa", gpu["dk"], dk), ("dL_demission", gpu["de"], de)):
        a = np.asarray(a, np.float64)
        par[key] = dict(l2_rel=float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)))
    ok = (par["J"]["max_rel"] <= 1e-5 and par["absorbed"]["max_rel"] <= 1e-5 and
          par["J"]["l1_rel"] <= 1e-5 and par["absorbed"]["l1_rel"] <= 1e-5 and
          par["totals_max_rel"] <= 1e-5 and
          all(par[key]["l2_rel"] <= 1e-5 for key in ("dL_dkappa", "dL_demission")))
    par["pass_1e-5"] = bool(ok)
    return par


def cpu_baseline(w: dict, n_updates: int, gpu_full: dict, gpu_run, threads: int = 0) -> dict:
    """The FP64 oracle on the host, timed over one step (forward and adjoint) of the
    same workload, and its element-wise comparison with the GPU.  A step larger than
    CPU_SAMPLE_UPDATES is sampled: the oracle then runs the same step for the first
    k directions only (same meshes, fields, passes and iterations), timed per update,
    and the GPU runs that sample too (untimed) for the comparison."""
    import numpy as np

    import oracle
    oracle.build()
    budget = CPU_SAMPLE_UPDATES
    if threads > 0:  # fewer threads: a proportionally smaller sample (same run time)
        budget *= min(1.0, threads / max(1, oracle.num_threads()))
        oracle.set_threads(threads)
    D = len(w["dirs"])
    k = sample_dirs(w, n_updates, budget)
    ws = w if k == D else dict(w, dirs=np.ascontiguousarray(w["dirs"][:k]))
    sample_updates = n_updates * k // D
    t0 = time.perf_counter()
    ref = oracle.forward(ws)
    gJ, gA = oracle.absorbed_loss_grads(ws)
    dk, de = oracle.adjoint(ws, gJ, gA)
    dt = time.perf_counter() - t0
    passes = n_updates // updates_per_pass(w)
    cores = oracle.num_threads()
    gpu = gpu_full if k == D else gpu_run(ws)
    return {"value": sample_updates / dt, "unit": "cell-direction updates/s", "cores": cores,
            "kind": "oracle", "host": host_cpu(),
            "sample": "%s of the same workload (%d updates: forward + adjoint, %d pass(es)), "
                      "FP64, %.1f s on %d OpenMP threads" % (
                          "one full step" if k == D else "one step over the first %d of %d "
                          "directions" % (k, D), sample_updates, passes, dt, cores),
            "parity_vs_gpu": dict(parity(gpu, ref, dk, de),
                                  sample="all directions of the timed step" if k == D else
                                  "the GPU on the oracle's %d-direction sample" % k)}


# ------------------------------------------------------------------ copy calibration
def copy_calibration(nbytes: int, reps: int) -> None:
    """A plain device copy of known size, for scaling the HBM counters."""
    import torch
    n = nbytes // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": reps}))


# ------------------------------------------------------------------ photoionisation workload
def hii_bench(args) -> int:
    """R-type HII region (hii_rtype lattice, 84 directions): one step is one time step,
    a forward sweep under the exponential law plus one chemistry step on the graphs
    built once.  Timed from the state after `warmup` steps of a neutral start."""
    import torch

    import paper_2207_12848_amd as sw
    from synth import workloads as W

    dev = torch.device("cuda:0")
    w = W.hii_rtype(args.hii_side, 84)
    p = dict(w["hii"])
    trec = 1.0 / (p["alpha_B"] * p["n_H"])
    p["dt_max"] = p["dt_max_trec"] * trec
    C = args.hii_side ** 3
    D = len(w["dirs"])
    meshes = [sw.upload_mesh(m, dev) for m in w["meshes"]]
    dag = sw.build_dag(meshes, w["dirs"])
    info = dag.info()
    e = torch.as_tensor(w["emission"]).to(dev).contiguous()
    t_w, y, _ = sw.evolve_ionisation(dag, e, p, 1e30, max_steps=max(args.warmup, 1))
    torch.cuda.synchronize()
    sw.profile_reset()
    sw.profile_enable(True)
    t0 = time.perf_counter()
    t_s, y, n = sw.evolve_ionisation(dag, e, p, 1e30, neutral=y, max_steps=args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sw.profile_enable(False)
    kt = sw.kernel_times()
    sw.profile_reset()
    ms = (t1 - t0) * 1e3 / max(n, 1)
    n_updates = C * D * n
    sizes = dict(C=C, H=6 * C, T=C * D, Eu=int(info["n_up_entries"]), Ed=int(info["n_down_entries"]),
                 G=1)
    per_kernel = {}
    for k, (cnt, tms) in kt.items():
        if cnt:
            b = byte_model(k, sizes)
            per_kernel[k] = dict(launches=cnt, ms_per_step=round(tms / n, 5),
                                 avg_launch_ms=round(tms / cnt, 5), alg_bytes_per_launch=b,
                                 alg_gbs=round(b / (tms / cnt * 1e-3) / 1e9, 2))
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_step"])
    pk = per_kernel[dom]
    roof = {"bound": "hbm", "achieved": pk["alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(pk["alg_gbs"] / HBM_PEAK_GBS, 5), "traffic": None, "kernel": dom,
            "bytes_per_launch": pk["alg_bytes_per_launch"], "avg_launch_ms": pk["avg_launch_ms"]}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import hii as OH
        k = 2
        c0 = time.perf_counter()
        OH.evolve(w, 1e30, max_steps=k)
        dt_cpu = time.perf_counter() - c0
        import oracle
        cpu = {"value": C * D * k / dt_cpu, "unit": "cell-direction updates/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "the first %d time steps of the same run (FP64 sweep + numpy chemistry), "
                         "%.1f s" % (k, dt_cpu)}
    line = {"metric": "cell-direction updates/s, photoionisation time steps (sweep + chemistry)",
            "value": n_updates / ((t1 - t0) if n else float("inf")), "unit": "cell-direction updates/s",
            "n_gpus": 1, "steps": n, "warmup": args.warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "hii_rtype", "cells": C, "directions": D, "groups": 1,
                       "law": "exp", "boundary": "vacuum", "simulated_time_trec": round(t_s / trec, 5)},
            "roofline": roof, "cpu_baseline": cpu, "kernels": per_kernel}
    print(json.dumps(line), flush=True)
    return 0


# ------------------------------------------------------------------ main
def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3_batched_groups", choices=WORKLOADS)
    ap.add_argument("--block", type=int, default=0, help="sweep workgroup size (0 = tuned)")
    ap.add_argument("--ring", type=int, default=0, help="LDS ring capacity (0 = tuned)")
    ap.add_argument("--pack", type=int, default=0,
                    help="groups swept together per work item, 1-4 (0 = automatic)")
    ap.add_argument("--hii-side", type=int, default=32,
                    help="lattice side of the hii_rtype workload")
    ap.add_argument("--law", default="upwind", choices=("upwind", "exp"),
                    help="cell law: first-order upwind balance or exponential attenuation")
    ap.add_argument("--scheme", default="area", choices=("area", "aligned"),
                    help="transport scheme: (a) area-weighted outflow or (b) the three most "
                         "aligned outflow faces")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="OpenMP threads of the oracle baseline (0 = all)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="pick block and ring with the library's autotuner before timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (PMC scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (the sweep would shard by direction "
              "with one all-reduce of J per pass); run with --gpus 1", file=sys.stderr)
        return 2
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, 5)
        return 0
    if args.workload == "hii_rtype":
        return hii_bench(args)

    import numpy as np
    import torch

    import paper_2207_12848_amd as sw

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")

    t0 = time.perf_counter()
    w = make_workload(args.workload)
    w["law"] = args.law
    w["scheme"] = args.scheme
    log("workload %s built in %.1f s" % (args.workload, time.perf_counter() - t0))
    G = int(w["G"])
    C = sum(len(m["cell_volume"]) for m in w["meshes"])
    D = len(w["dirs"])
    H = sum(len(m["face_nbr"]) for m in w["meshes"])
    meshes = [sw.upload_mesh(m, dev) for m in w["meshes"]]
    kappa = torch.as_tensor(w["kappa"]).to(dev).contiguous()
    emission = torch.as_tensor(w["emission"]).to(dev).contiguous()
    gJ = torch.zeros((C, G), dtype=torch.float32, device=dev)
    gA = torch.full((C, G), 1.0 / (4.0 * math.pi), dtype=torch.float32, device=dev)
    fo = fwd_opts(w, "batched", args.block, args.ring, args.pack)

    # validate the mesh once; the timed steps rebuild the graphs without re-checking it
    dag0 = sw.build_dag(meshes, w["dirs"], validate=True, scheme=args.scheme)
    info = dag0.info()
    tuned = None
    if args.tune:
        tuned = sw.tune(dag0, kappa, emission, reps=2, **fwd_opts(w))
        fo["block"], fo["ring"], fo["pack"] = tuned["block"], tuned["ring"], tuned["pack"]
        log("tuned launch shape: %s" % tuned)
    dag0.close()

    def step(form="batched", dirs=None):
        """build + forward (saving for the adjoint) + adjoint of the absorbed-photon loss"""
        o = dict(fo, form=form)
        dag = sw.build_dag(meshes, w["dirs"] if dirs is None else dirs, validate=False,
                           scheme=args.scheme)
        J, A, tot, saved = sw.forward(dag, kappa, emission, save_for_adjoint=True, **o)
        dk, de = sw.adjoint(dag, kappa, emission, saved, gJ, gA, **o)
        return dag, J, A, tot, dk, de

    # every pass of the forward is a sweep of all C * D * G updates; the adjoint
    # sweeps every pass again in reverse (its recomputed passes are not counted)
    passes_fwd = int(fo["n_pbc"]) * int(fo["n_scat"])
    passes_adj = passes_fwd
    n_updates = C * D * G * (passes_fwd + passes_adj)

    for i in range(args.warmup):
        out = step()
        out[0].close()
        log("warmup %d done" % i)
    torch.cuda.synchronize()

    sw.profile_reset()
    sw.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step()
        if i + 1 < args.steps:
            out[0].close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sw.profile_enable(False)
    kt = sw.kernel_times()
    sw.profile_reset()
    ms = (t1 - t0) * 1e3 / max(args.steps, 1)
    value = n_updates / (ms * 1e-3)
    log("timed %d steps: %.3f ms/step" % (args.steps, ms))

    dag, J, A, tot, dk, de = out
    gpu = dict(J=J.cpu().numpy(), absorbed=A.cpu().numpy(), totals=tot.cpu().numpy(),
               dk=None if dk is None else dk.cpu().numpy(),
               de=None if de is None else de.cpu().numpy())
    dag.close()

    # roofline of the dominant kernel (largest share of the timed region)
    sizes = dict(C=C, H=H, T=C * D, Eu=int(info["n_up_entries"]), Ed=int(info["n_down_entries"]),
                 G=G)
    per_kernel = {}
    for k, (n, tms) in kt.items():
        if n == 0:
            continue
        b = byte_model(k, sizes)
        per_kernel[k] = dict(launches=n, ms_per_step=tms / args.steps, avg_launch_ms=tms / n,
                             alg_bytes_per_launch=b,
                             alg_gbs=b / (tms / n * 1e-3) / 1e9)
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_step"])
    pk = per_kernel[dom]
    traffic = read_traffic(dom, args.workload)
    roof = {"bound": "hbm", "achieved": round(pk["alg_gbs"], 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(pk["alg_gbs"] / HBM_PEAK_GBS, 5), "traffic": traffic,
            "kernel": dom, "bytes_per_launch": pk["alg_bytes_per_launch"],
            "avg_launch_ms": round(pk["avg_launch_ms"], 4)}

    def run_sample(ws):
        """The batched GPU step on a direction sample (untimed), as numpy outputs."""
        dag, J, A, tot, dk, de = step(dirs=ws["dirs"])
        torch.cuda.synchronize()
        r = dict(J=J.cpu().numpy(), absorbed=A.cpu().numpy(), totals=tot.cpu().numpy(),
                 dk=dk.cpu().numpy(), de=de.cpu().numpy())
        dag.close()
        return r

    # plain per-(mesh, direction, group) form of the same step, for comparison: on the
    # first few directions when the whole step would take long in this form (its
    # launches run one after another, so its time per update does not depend on D)
    plain = None
    if not args.no_plain:
        kp = D if n_updates <= PLAIN_SAMPLE_UPDATES else max(1, int(D * PLAIN_SAMPLE_UPDATES / n_updates))
        pdirs = np.ascontiguousarray(w["dirs"][:kp])
        out = step("plain", dirs=pdirs)
        out[0].close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = step("plain", dirs=pdirs)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) * 1e3
        out[0].close()
        pupd = n_updates * kp // D
        pv = pupd / (pms * 1e-3)
        plain = {"value": pv, "ms_per_step": round(pms, 3), "directions": kp,
                 "updates_per_step": pupd, "batched_speedup": round(value / pv, 2),
                 "sample": "one step over all directions" if kp == D else
                           "one step over the first %d of %d directions" % (kp, D)}
        log("plain form: %.3f ms/step over %d directions" % (pms, kp))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, n_updates, gpu, run_sample, args.cpu_threads)
        log("cpu baseline: %.3g updates/s on %d threads" % (cpu["value"], cpu["cores"]))

    depth_max = int(info["max_depth"])
    def kms(*ks):
        return sum(per_kernel.get(k, {}).get("ms_per_step", 0.0) for k in ks)
    line = {
        "metric": "cell-direction updates/s, fwd+adjoint, batched vs plain, rel err <=1e-5 vs FP64",
        "value": value,
        "unit": "cell-direction updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": C, "directions": D, "groups": G,
                   "meshes": len(w["meshes"]), "boundary": w.get("boundary", "vacuum"),
                   "n_pbc": fo["n_pbc"], "n_scat": fo["n_scat"], "albedo": fo["albedo"],
                   "law": fo["law"], "scheme": args.scheme,
                   "adjoint": True, "updates_per_step": n_updates, "form": "batched",
                   "block": fo["block"] or "default", "ring": fo["ring"] or "default",
                   "pack": fo["pack"] or "auto"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain": plain,
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in per_kernel.items()},
        "dag": {"depth_max": depth_max, "depth_min": int(info["min_depth"]),
                "depth_mean": round(float(info["mean_depth"]), 1),
                "up_entries_per_task": round(sizes["Eu"] / sizes["T"], 3),
                "sweep_us_per_level_fwd": round(
                    per_kernel.get("sweep_fwd", {}).get("avg_launch_ms", 0.0) * 1e3 /
                    max(depth_max, 1), 3)},
        "phase_ms_per_step": {"build": round(kms("count", "kahn", "fill"), 4),
                              "forward": round(kms("prep", "sweep_fwd", "reduce"), 4),
                              "adjoint": round(kms("sweep_adj"), 4)},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
