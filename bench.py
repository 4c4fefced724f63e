#!/usr/bin/env python3
"""Benchmark of the graph-based S_N transport sweep on one MI355X.

Metric: DOF-direction updates per second of one full lagged sweep (every
level of the combined schedule, the scattering source and the scalar-flux
reduction), E*n*D / t_sweep, with all inputs resident in HBM; and the time to
a 1e-8 residual of source iteration with and without the learned correction.
Default workload: 3D 48^3 Q2 curved mesh (warp 0.05), DG p=2, S12 (168
directions), sigma_t in {1, 100} at random (seed 100), c = 0.99, q = 1,
vacuum; seeded synthetic inputs.

The line also carries:
  * roofline -- the algorithmic work of the method per (element, direction)
    pair (element assembly, face blocks, LU and the two triangular solves;
    geometry read once per element, traces written and read once) over the
    sweep kernel's average launch time (HIP events around every launch in a
    second timed pass), against the FP64 vector peak or HBM, whichever
    bounds that work; the cached-inverse byte stream the kernel actually
    reads is reported beside it (``inverse_stream``);
  * learned_vs_plain -- plain source iteration and the learned correction to
    1e-8 on the benchmarked problem (held out: the network is trained on
    other seeds of the same family first; training reported separately);
  * cpu_baseline -- the CPU oracle on a bounded sample of the same workload,
    with all host threads and with one;
  * secondary -- the 2D 128x128 Q3 S8 cyclic workload's sweep rate.

  python bench.py [--steps K] [--warmup W] [--workload c5|c1|c2|c3|c4]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBS = 8000.0
METRIC = "DOF-direction updates/s per sweep; time to 1e-8 residual, learned vs plain SI"
# HBM bytes per launch of the timed kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes, scaled by a copy kernel of known size (fetch x2.000,
# write x1.000), averaged over the launches of a sweep; the profiles/ files
# named after each kernel and workload hold the counts.  Only valid for the
# kernel build it was measured on: drop an entry when the kernel changes.
MEASURED_TRAFFIC = {("sweep_persistent_dpp<2,3,inv,nt>", "c2", "fp64"): 1.902e9,
                    ("sweep_persistent_dpp<2,3,inv,nt,f32>", "c2", "mixed"): 1.247e9,
                    ("sweep_level_inv<3,2>", "c5", "fp64"): 4.701e8,
                    ("sweep_level_inv<3,2,f32>", "c5", "mixed"): 3.102e8,
                    ("sweep_level_inv<3,2>", "c3", "fp64"): 1.376e8}
DESCRIPTIONS = {
    "c1": "2D 8x8 Q2 curved (warp 0.05), p=1, S4 (12 dirs), sigma_t=1, c=0.5, q=1, vacuum",
    "c2": "2D 128x128 Q3 curved (warp 0.3 h, 4-element wavelength, cyclic sweep graphs), p=3, "
          "S8 (40 dirs), sigma_t=1, c=0.8, q=1, vacuum",
    "c3": "3D 32^3 Q2 curved (warp 0.05), p=2, S8 (80 dirs), checkerboard sigma_t {1,10}, c=0.9, "
          "q=1 in the central 8^3 block, vacuum",
    "c5": "3D 48^3 Q2 curved (warp 0.05), p=2, S12 (168 dirs), random sigma_t {1,100} (seed 100), "
          "c=0.99, q=1, vacuum",
    "c4": "batch of 64 independent 2D problems (seed 0): m^2 Q2 meshes m in [16,96], p in {1,2,3}, "
          "S4-S12, sigma_t log-uniform [0.1,10], c uniform [0,0.95], q=1, vacuum; one hipGraph "
          "replay per batch sweep, schedule per (dim, p) class chosen by the autotuner",
}


def work_model(dim: int, p: int):
    """Algorithmic work of one (element, direction) update of the method:
    LU of the n x n element system (2/3 n^3) and the two triangular solves
    (2 n^2); assembly of sigma_t M - sum_i Omega_i K_i from the
    direction-independent matrices (2 (d+1) n^2) and of the scattering and
    source load M phi (2 n^2); face blocks from the normal moments
    (4 d (d+1) nf^2).  Returns (flops per pair, n, nf)."""
    n = (p + 1) ** dim
    nf = (p + 1) ** (dim - 1)
    flops = (2.0 / 3.0) * n ** 3 + 2 * n ** 2 + 2 * (dim + 1) * n ** 2 + 2 * n ** 2 + 4 * dim * (dim + 1) * nf ** 2
    return flops, n, nf


def algorithmic_bytes(dim: int, p: int, E: int, D: int, F_int: int) -> float:
    """HBM bytes the method must move per sweep: the direction-independent
    geometry (M and the d matrices K_i, FP64) once per element, every
    interior trace written once and read once (nf FP64 values per interior
    face and direction), and the scalar flux read and written."""
    n = (p + 1) ** dim
    nf = (p + 1) ** (dim - 1)
    return 8.0 * (E * (dim + 1) * n * n + 2.0 * F_int * D * nf + 2.0 * E * n)


def interior_faces(nx) -> int:
    nx = list(nx)
    tot = 0
    for a in range(len(nx)):
        prod = 1
        for b in range(len(nx)):
            prod *= (nx[b] - 1) if b == a else nx[b]
        tot += prod
    return tot


def inverse_stream_bytes_per_pair(dim: int, p: int, f32: bool = False) -> float:
    """Bytes the cached-inverse kernels read or write per pair: its A^{-1}
    (n^2 doubles, or in mixed precision n * 4 ceil(n/4) floats), its new
    angular flux (n) and the upwind traces of its d inflow faces (nf each)."""
    n = (p + 1) ** dim
    nf = (p + 1) ** (dim - 1)
    inv = 4.0 * n * 4 * ((n + 3) // 4) if f32 else 8.0 * n * n
    return inv + 8.0 * (n + dim * nf)


def host_cpu():
    """(cores available to this process, CPU model name)."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return len(os.sched_getaffinity(0)), model


def cpu_baseline(wp, block: int = None, n_dirs_sample: int = None):
    """The oracle's lagged sweep timed on a bounded sample of the workload
    (CPU baseline, not tuned): for 3D workloads the corner block of
    block^3 elements of the same mesh and materials, all directions unless
    n_dirs_sample is given; the setup (geometry, faces, graphs) is not timed,
    as on the GPU.  Timed twice: with the host's BLAS threads and with one."""
    import numpy as np
    import workloads as W
    from oracle.discretization import Discretization
    from oracle.quadrature import level_symmetric
    from oracle.sweep import build_graphs, sweep
    sample = wp if block is None else W.corner_block(wp, block)
    om, w = level_symmetric(sample.sn_order, sample.dim)
    sel = np.arange(len(w)) if n_dirs_sample is None else \
        np.linspace(0, len(w) - 1, min(n_dirs_sample, len(w))).round().astype(int)
    disc = Discretization(sample, omega=om[sel], w=w[sel])
    gs = build_graphs(disc)
    rng = np.random.default_rng(5)
    phi0 = rng.uniform(0.0, 2.0, (disc.E, disc.n))
    psi0 = rng.uniform(0.0, 0.2, (disc.D, disc.E, disc.n))
    cores, model = host_cpu()
    blas = None
    runs = {}
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        blas = max([1] + [int(i.get("num_threads", 1)) for i in threadpool_info()])
    except Exception:
        threadpool_limits = None
    for label in ("all", "serial"):
        if label == "serial" and threadpool_limits is None:
            continue
        t0 = time.perf_counter()
        if label == "serial":
            with threadpool_limits(limits=1):
                sweep(disc, gs, phi0, psi0)
        else:
            sweep(disc, gs, phi0, psi0)
        runs[label] = time.perf_counter() - t0
    dof_dir = disc.E * disc.n * disc.D
    where = f"the {block}^{sample.dim} corner block of the mesh" if block is not None else "the full mesh"
    out = {"value": dof_dir / runs["all"], "unit": "DOF-dir/s", "cores": blas or 1, "kind": "oracle",
           "sample": f"1 lagged sweep of {len(sel)} of {len(w)} directions on {where} ({disc.E} elements, "
                     f"{dof_dir} DOF-dir) from seeded fluxes, {runs['all']:.2f} s",
           "host_cores": cores, "cpu_model": model}
    if "serial" in runs:
        out["serial"] = {"value": dof_dir / runs["serial"], "cores": 1, "seconds": round(runs["serial"], 2)}
    return out


def kernel_name(wp, sched: int, inv: int, tile: int) -> str:
    if sched == 1:
        if wp.dim == 2 and wp.p != 2:
            nt = ",nt" if inv and tile > 0 else ""
            f32 = ",f32" if inv == 2 else ""
            return f"sweep_persistent_dpp<{wp.dim},{wp.p}{',inv' if inv else ''}{nt}{f32}>"
        if inv:
            if wp.dim == 2:
                return f"sweep_persistent_lds2d<{wp.p}{',f32' if inv == 2 else ''}>"
            return f"sweep_persistent_inv<{wp.dim},{wp.p}>"
        return f"sweep_persistent_fp64<{wp.dim},{wp.p}>"
    if inv == 2:
        return f"sweep_level_inv<{wp.dim},{wp.p},f32>"
    return f"sweep_level_inv<{wp.dim},{wp.p}>" if inv else f"sweep_level_fp64<{wp.dim},{wp.p}>"


def time_sweeps(P, steps: int, warmup: int):
    """Whole-sweep time (ms) between HIP events on the problem's stream, then
    a second pass with HIP events around every sweep-kernel launch.
    Returns (ms per sweep, launches per sweep, summed kernel ms per sweep)."""
    import torch
    E, n = P.E, P.n
    phi = torch.zeros(E * n, dtype=torch.float64, device="cuda")
    out = torch.empty_like(phi)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        P.sweep(phi, out)
        phi, out = out, phi
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        P.sweep(phi, out)
        phi, out = out, phi
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    P.profile_enable(True)
    for _ in range(steps):
        P.sweep(phi, out)
        phi, out = out, phi
    launches, kernel_ms = P.profile_read()
    P.profile_enable(False)
    P.synchronize()
    return ms, launches / steps, kernel_ms / steps


def sweep_line(P, wp, name: str, sched: int, prec: int, steps: int, warmup: int):
    """Sweep rate and roofline of one problem (dict parts of the JSON line)."""
    info = P.info()
    E, n, D = P.E, P.n, P.D
    ms, launches, kernel_ms = time_sweeps(P, steps, warmup)
    inv = bool(info["cached_inverse"])
    partial = inv and info["cached_dirs"] < D
    kname = kernel_name(wp, sched, info["cached_inverse"], info["tile"])
    if partial:
        kname += " + " + kernel_name(wp, sched, 0, info["tile"])
    flops_pair, _, _ = work_model(wp.dim, wp.p)
    flops = flops_pair * E * D
    nbytes = algorithmic_bytes(wp.dim, wp.p, E, D, interior_faces(wp.nx))
    t_alu = flops / (FP64_VECTOR_PEAK_TFLOPS * 1e12)
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    avg_launch_s = kernel_ms / launches * 1e-3
    if t_alu >= t_hbm:
        achieved = flops / launches / avg_launch_s / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 5)}
    else:
        achieved = nbytes / launches / avg_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5)}
    traffic = None if partial else MEASURED_TRAFFIC.get((kname, name, "fp64" if prec == 0 else "mixed"))
    roof.update({"traffic": traffic, "kernel": kname,
                 "algorithmic_flops_per_sweep": flops, "algorithmic_bytes_per_sweep": nbytes,
                 "roofline_ms_per_sweep": round(max(t_alu, t_hbm) * 1e3, 4),
                 "avg_launch_us": round(avg_launch_s * 1e6, 3), "launches_per_sweep": launches,
                 "kernel_share_of_step": round(kernel_ms / ms, 4)})
    if inv and not partial:
        sb = inverse_stream_bytes_per_pair(wp.dim, wp.p, f32=info["cached_inverse"] == 2) * E * D + 8.0 * E * n
        gbs = sb / launches / avg_launch_s / 1e9
        roof["inverse_stream"] = {"bytes_per_sweep": sb, "achieved_gbs": round(gbs, 1),
                                  "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 5),
                                  "traffic_over_stream": round(traffic * launches / sb, 3) if traffic else None}
    return {"value": E * n * D / (ms * 1e-3), "ms_per_step": round(ms, 5), "roofline": roof,
            "config": {"workload": DESCRIPTIONS[name], "elements": E, "dofs_per_element": n, "directions": D,
                       "levels": info["n_levels_total"], "lagged_edges": info["n_removed_total"],
                       "kink_face_dirs": info["n_kink_faces_total"], "cached_inverse": inv,
                       "cached_dirs": info["cached_dirs"],
                       "schedule": "persistent" if sched == 1 else "levels",
                       "precision": "fp64" if prec == 0 else "mixed"}}


def bench_batch(args):
    """Batched sweep of the 64-problem workload: value = summed E*n*D over
    the batch / time of one batch sweep (graph replay)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1810_11080_amd import Batch, Context, Problem

    wps = W.c4()
    ctx = Context(device=0)
    t0 = time.perf_counter()
    problems = [Problem.from_workload(ctx, wp) for wp in wps]
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    B = Batch(ctx, problems, schedule={"auto": 0, "persistent": 1, "levels": 2}[args.schedule], use_graph=True)
    tune_s = time.perf_counter() - t0
    ins = [torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda") for P in problems]
    outs = [torch.empty_like(t) for t in ins]
    for _ in range(args.warmup):
        B.sweep(ins, outs)
        ins, outs = outs, ins
    B.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        B.sweep(ins, outs)
        ins, outs = outs, ins
    ev1.record(stream)
    B.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    dof_dir = sum(P.E * P.n * P.D for P in problems)
    # the method's algorithmic work summed over the problems (same model as
    # the single-problem line); the batch is timed as a whole replay
    flops = sum(work_model(wp.dim, wp.p)[0] * P.E * P.D for wp, P in zip(wps, problems))
    nbytes = sum(algorithmic_bytes(wp.dim, wp.p, P.E, P.D, interior_faces(wp.nx)) for wp, P in zip(wps, problems))
    classes = B.classes()
    t_alu = flops / (FP64_VECTOR_PEAK_TFLOPS * 1e12)
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    kname = "whole batch sweep (graph replay: source, fill, class sweeps, scalar flux)"
    if t_alu >= t_hbm:
        achieved = flops / (ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 5)}
    else:
        achieved = nbytes / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5)}
    roof.update({"traffic": None, "kernel": kname, "algorithmic_flops_per_sweep": flops,
                 "algorithmic_bytes_per_sweep": nbytes, "roofline_ms_per_sweep": round(max(t_alu, t_hbm) * 1e3, 4)})
    line = {
        "metric": METRIC,
        "value": dof_dir / (ms * 1e-3),
        "unit": "DOF-dir/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS["c4"], "problems": len(problems), "dof_dir_per_sweep": dof_dir,
                   "setup_s": round(setup_s, 2), "tune_s": round(tune_s, 2),
                   "classes": [{"p": c["dg_order"], "problems": c["n_problems"], "levels": c["n_levels"],
                                "schedule": ("persistent" + (" tiled" if c["tiled"] else "")) if c["persistent"] else "levels",
                                "blocks": c["blocks"], "tuned_ms": [round(x, 3) for x in c["tuned_ms"]]}
                               for c in classes]},
        "roofline": roof,
        "cpu_baseline": None,
    }
    print(json.dumps(line))


def note(msg: str):
    print(msg, file=sys.stderr, flush=True)


def train_correction(ctx, family, train_seeds, steps: int, stride: int, tol_train: float):
    """Trains the learned correction (widths 16/32/32) on plain-SI pairs of
    the training seeds of a problem family: every `stride`-th iteration of a
    solve from zero to tol_train gives a pair.  Each training problem is
    freed before the next one is built.  Returns (net, training report)."""
    import torch
    from paper_1810_11080_amd import Net, Problem
    from paper_1810_11080_amd import learn as L
    t0 = time.perf_counter()
    Xs, Ts, grid = [], [], None
    for seed in train_seeds:
        P = Problem.from_workload(ctx, family(seed))
        grid = L.element_grid(P)
        kept, star, its = L.plain_trajectory(P, tol=tol_train, max_iters=50000, sample=lambda l: l % stride == 0)
        X, T = L.make_pairs(P, kept, star)
        Xs.append(X)
        Ts.append(T)
        note(f"training seed {seed}: {its} plain sweeps, {len(kept)} pairs, {time.perf_counter() - t0:.1f} s")
        del kept, star
        P.close()
        del P
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    del Xs, Ts
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    net = Net(ctx, widths=(16, 32, 32), seed=0)
    t0 = time.perf_counter()
    losses = L.train(net, grid, X, T, steps=steps, batch=8, lr=2e-3, lr_final=1e-4)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    note(f"trained {steps} steps in {train_s:.1f} s, loss {losses[:10].mean():.4g} -> {losses[-100:].mean():.4g}")
    rep = {"seeds": list(train_seeds), "pairs": int(X.shape[0]), "tol": tol_train, "stride": stride,
           "data_s": round(data_s, 2), "train_s": round(train_s, 2), "steps": steps, "batch": 8,
           "loss_first": float(losses[:10].mean()), "loss_last": float(losses[-100:].mean())}
    return net, rep


def compare_solves(P, net, every: int, tol: float = 1e-8, max_iters: int = 50000):
    """Source iteration from zero to tol, plain and with the learned
    correction, on the same problem.  Returns the two reports."""
    import torch
    out = {}
    for name, pre in (("plain", None), ("learned", net)):
        P.reset()
        phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
        rep = P.solve(phi, tol=tol, max_iters=max_iters, precond=pre, precond_every=every,
                      raise_on_not_converged=False)
        out[name] = {"seconds": round(rep["seconds"], 4), "sweeps": rep["iterations"],
                     "residual": rep["residual"]}
        if pre is not None:
            out[name].update(corrections=rep["n_corrected"], rejected=rep["n_rejected"])
        note(f"{name}: {out[name]}")
    return out


def learned_block(runs, training, every, eval_desc, params):
    plain = sum(r["plain"]["seconds"] for r in runs) / len(runs)
    learned = sum(r["learned"]["seconds"] for r in runs) / len(runs)
    saved = plain - learned
    training = dict(training, break_even_solves=round((training["data_s"] + training["train_s"]) / saved, 1)
                    if saved > 0 else None)
    return {"workload": eval_desc, "tol": 1e-8, "precond_every": every, "params": params,
            "time_plain_s": round(plain, 4), "time_learned_s": round(learned, 4),
            "speedup": round(plain / learned, 3), "runs": runs, "training": training}


def lagged_face_fraction(P, P_face) -> float:
    """Share of the face-weighted coupling that a problem's cut lags: the sum
    over its removed edges of the face weights (taken from P_face, the same
    mesh built with face weighting) over the sum of all face weights."""
    import numpy as np
    lag = tot = 0
    for d in range(P.D):
        up, down, w = P_face.edges(d)
        wd = {(int(u), int(v)): int(x) for u, v, x in zip(up, down, w)}
        tot += int(np.sum(w))
        rd, ru = P.removed_edges(d)
        lag += sum(wd[(int(u), int(v))] for u, v in zip(ru, rd))
    return lag / max(tot, 1)


def weighting_study(tol: float = 1e-8, max_iters: int = 20000):
    """Unity vs face vs sigma-inverse-face edge weights on meshes whose sweep
    graphs have cycles (eq. graphWeight and the cycle-cutting of section 3):
    removed edges, largest SCC, levels, share of the face coupling that is
    lagged, and plain source iteration to `tol` on the GPU."""
    import dataclasses
    import torch
    import workloads as W
    from paper_1810_11080_amd import Context, Problem
    ctx = Context(0)
    host = Context(-1)
    cases = [W.standin_2d(16, 21), W.standin_2d(32, 42), W.standin_3d(), W.annulus_quarter(9, 15, 3, 4),
             W.annulus_quarter(18, 30, 3, 4), W.cyclic_2d(32, 4, 0.9, 2, 8), W.cyclic_2d(64, 8, 0.9, 2, 8), W.c2()]
    names = {0: "unity", 1: "face", 2: "siginvface"}
    rows = []
    for wp in cases:
        P_face = Problem.from_workload(host, dataclasses.replace(wp, weighting=1))
        for wgt in (0, 1, 2):
            P = Problem.from_workload(ctx, dataclasses.replace(wp, weighting=wgt))
            st = [P.graph_stats(d) for d in range(P.D)]
            frac = lagged_face_fraction(P, P_face)
            phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
            rep = P.solve(phi, tol=tol, max_iters=max_iters)
            row = {"case": wp.name, "weighting": names[wgt], "E": P.E, "D": P.D,
                   "removed": int(sum(x["n_removed"] for x in st)),
                   "max_scc": int(max(x["max_scc"] for x in st)),
                   "levels_max": int(max(x["n_levels"] for x in st)),
                   "lagged_face_coupling": round(frac, 6),
                   "iterations": int(rep["iterations"]), "solve_s": round(rep["seconds"], 4)}
            rows.append(row)
            print("| {case} | {weighting} | {removed} | {max_scc} | {levels_max} | {lagged_face_coupling:.4%} | "
                  "{iterations} | {solve_s} |".format(**row), file=sys.stderr, flush=True)
            P.close()
        P_face.close()
    return rows


def mms_error(ctx, wp, tol: float = 1e-13, extra: int = 4):
    """Solve the manufactured problem of eq. psiAnnularMMS on the mesh and
    materials of wp with the library (nodal source and tabulated incident
    flux evaluated at the library's DG node positions); returns the scalar
    flux L2 error against the closed form (Gauss rule with `extra` points per
    axis beyond the element-matrix rule), the unknowns per direction and the
    solve report."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1810_11080_amd import Problem
    P = Problem.from_workload(ctx, wp)
    om, w = P.quadrature()
    st = np.repeat(wp.sigma_t, P.n).reshape(P.E, P.n)
    ss = np.repeat(wp.sigma_s, P.n).reshape(P.E, P.n)
    q, psi_exact, _ = W.mms_annular(P.node_coordinates(), om, w, st, ss)
    P.set_source(q, bc_kind=W.TABULATED, psi_inc_tab=psi_exact)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    rep = P.solve(phi, tol=tol, max_iters=2000)
    x, wd, basis = P.volume_rule(extra=extra)
    _, _, phi_exact = W.mms_annular(x, om, w, 0.0, 0.0)
    ph = phi.cpu().numpy().reshape(P.E, P.n) @ basis.T
    err = float(np.sqrt(np.sum(wd * (ph - phi_exact) ** 2)))
    out = (err, P.E * P.n, rep)
    P.close()
    return out


def ho_vs_lo(levels=(1, 2, 4)):
    """High-order vs straightened low-order accuracy on the quarter annulus
    (curved boundaries, the three material rings of the nested-annuli
    problem), manufactured solution of eq. psiAnnularMMS, S4: Q3 meshes with
    cubic DG (9k x 15k elements) against their straightening into linear
    elements with linear DG (N_ref = 3: 27k x 45k elements), the format of
    the paper's L2-error table."""
    import workloads as W
    from paper_1810_11080_amd import Context
    ctx = Context(0)
    rows = []
    for k in levels:
        ho = W.annulus_quarter(9 * k, 15 * k, 3, 4)
        for name, wp in (("HO (Q3 mesh, p=3)", ho), ("straightened (Q1 mesh, p=1)", W.straightened(ho, p=1))):
            err, unknowns, rep = mms_error(ctx, wp)
            row = {"mesh": name, "refinement": k, "elements": int(wp.n_elements), "unknowns": int(unknowns),
                   "l2_error": err, "sweeps": rep["iterations"], "solve_s": round(rep["seconds"], 4)}
            rows.append(row)
            note("| {mesh} | {refinement} | {elements} | {unknowns} | {l2_error:.4e} | {sweeps} |".format(**row))
    return rows


def element_study(steps: int = 20, warmup: int = 3):
    """Sweep rates of curved triangles (the simplicial elements) against
    quadrilaterals on the same closed annulus (r in [1, 2], cubic maps, p = 2,
    S8): 96 x 384 cells as 73,728 triangles (n = 6) or 36,864 quads (n = 9),
    level schedule and persistent kernels, with cached inverses and
    assembled per sweep."""
    import workloads as W
    from paper_1810_11080_amd import Context, Problem
    ctx = Context(0)
    rows = []
    meshes = (("triangles P2 (Q3 map)", W.tri_annulus(nr=96, nt=384, r=3, p=2, sn_order=8, seed=1)),
              ("quads Q2 (Q3 map)", W.annulus_full(nr=96, nt=384, p=2, sn_order=8, r=3, seed=1)))
    for label, wp in meshes:
        for sched, cache, cname in ((2, 1, "levels, cached inverse"), (2, 2, "levels, assembled"),
                                    (1, 1, "persistent, cached inverse"), (1, 2, "persistent, assembled")):
            t0 = time.perf_counter()
            P = Problem.from_workload(ctx, wp, schedule=sched, cache_inverse=cache)
            setup = time.perf_counter() - t0
            ms, launches, kernel_ms = time_sweeps(P, steps, warmup)
            rate = P.E * P.n * P.D / (ms * 1e-3)
            row = {"mesh": label, "elements": int(P.E), "n": int(P.n), "directions": int(P.D), "path": cname,
                   "ms_per_sweep": round(ms, 4), "launches": launches, "dof_dir_per_s": rate,
                   "pairs_per_s": P.E * P.D / (ms * 1e-3), "setup_s": round(setup, 2)}
            rows.append(row)
            note("| {mesh} | {path} | {elements} | {n} | {ms_per_sweep} | {dof_dir_per_s:.3e} | "
                 "{pairs_per_s:.3e} |".format(**row))
            del P
    return rows


def learned_study(train_steps: int, eval_seeds=(100, 101, 102, 103), every: int = 40):
    """The learned correction on the 48^3 S12 family: trained on seeds 0 and
    1 (as the default line), then plain vs learned source iteration to 1e-8
    on each held-out seed, and an ablation with the same network untrained
    (its initial weights) on the first held-out seed."""
    import torch
    import workloads as W
    from paper_1810_11080_amd import Context, Net, Problem
    ctx = Context(device=0)
    net, training = train_correction(ctx, lambda seed: W.c5(seed=seed), (0, 1), train_steps, 10, 1e-10)
    untrained = Net(ctx, widths=(16, 32, 32), seed=0)
    runs, ablation = [], None
    for seed in eval_seeds:
        P = Problem.from_workload(ctx, W.c5(seed=seed))
        note(f"seed {seed}: problem built")
        r = compare_solves(P, net, every)
        runs.append(dict(seed=seed, **r))
        if ablation is None:
            P.reset()
            phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
            rep = P.solve(phi, tol=1e-8, max_iters=50000, precond=untrained, precond_every=every,
                          raise_on_not_converged=False)
            ablation = {"seed": seed, "seconds": round(rep["seconds"], 4), "sweeps": rep["iterations"],
                        "residual": rep["residual"], "corrections": rep["n_corrected"],
                        "rejected": rep["n_rejected"]}
            note(f"untrained network: {ablation}")
        P.close()
        del P
        torch.cuda.synchronize()
    block = learned_block(runs, training, every, DESCRIPTIONS["c5"].replace(" (seed 100)", "") +
                          "; network trained on seeds 0 and 1", net.n_params)
    block["untrained_network"] = ablation
    return block


def calibrate_copy(nbytes: int = 1 << 30, reps: int = 3):
    """A plain streaming kernel of known traffic (read nbytes, write nbytes):
    the reference for scaling HBM counter readings to bytes."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "elementwise copy kernel", "read_bytes": nbytes, "write_bytes": nbytes,
                      "launches": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5", choices=sorted(DESCRIPTIONS),
                    help="c5 (default): the 48^3 S12 benchmark; c4: the 64-problem batch")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--schedule", default="auto", choices=["auto", "persistent", "levels"])
    ap.add_argument("--cache-inverse", default="auto", choices=["auto", "on", "off"],
                    help="keep each pair's A^{-1} on the device (factored once at setup)")
    ap.add_argument("--cache-budget", type=float, default=0.0,
                    help="GB the cached inverses may take under auto (0: half the free memory; less than all of "
                         "them caches the first directions that fit)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training and the learned-vs-plain comparison (plain solve only)")
    ap.add_argument("--no-solve", action="store_true", help="no solves at all")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 2D cyclic secondary line")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a copy kernel of known size (HBM counter calibration)")
    ap.add_argument("--weighting-study", action="store_true",
                    help="only the unity / face / sigma-inverse-face weighting comparison")
    ap.add_argument("--ho-vs-lo", action="store_true",
                    help="only the high-order vs straightened low-order manufactured-solution comparison")
    ap.add_argument("--element-study", action="store_true",
                    help="only the sweep rates of curved triangles vs quads on one closed annulus")
    ap.add_argument("--learned-study", action="store_true",
                    help="only the learned correction on 48^3 S12: held-out seeds 100-103 and an untrained ablation")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(directions would be sharded across GPUs with one scalar-flux all-reduce "
              "per iteration; not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1810_11080_amd import Context, Problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.weighting_study:
        print(json.dumps({"weighting_study": weighting_study()}))
        return
    if args.ho_vs_lo:
        print(json.dumps({"ho_vs_lo": ho_vs_lo()}))
        return
    if args.learned_study:
        print(json.dumps({"learned_study": learned_study(args.train_steps)}))
        return
    if args.element_study:
        print(json.dumps({"element_study": element_study()}))
        return
    if args.workload == "c4":
        bench_batch(args)
        return
    ctx = Context(device=0)
    name = args.workload
    prec = 0 if args.precision == "fp64" else 1
    net = training = None
    every = 40
    if name == "c5" and not (args.no_learned or args.no_solve):
        # training first, so that only one 48^3 problem holds device memory
        # at a time (each caches 108 GB of element inverses)
        net, training = train_correction(ctx, lambda seed: W.c5(seed=seed), (0, 1), args.train_steps, 10, 1e-10)
    wp = W.CONFIGS[name]()
    t0 = time.perf_counter()
    sched = {"auto": 0, "persistent": 1, "levels": 2}[args.schedule]
    cache = {"auto": 0, "on": 1, "off": 2}[args.cache_inverse]
    P = Problem.from_workload(ctx, wp, precision=prec, schedule=sched, cache_inverse=cache,
                              cache_budget=args.cache_budget * 1e9)
    sched = P.info()["schedule"]      # the library's choice under "auto"
    setup_s = time.perf_counter() - t0
    note(f"{name}: setup {setup_s:.1f} s")
    main_line = sweep_line(P, wp, name, sched, prec, args.steps, args.warmup)
    main_line["config"]["setup_s"] = round(setup_s, 2)
    note(f"{name}: {main_line['ms_per_step']} ms per sweep")

    solve = learned = None
    if not args.no_solve:
        runs = compare_solves(P, net, every) if net is not None else None
        if runs is not None:
            learned = learned_block([dict(seed=100, **runs)], training, every,
                                    DESCRIPTIONS[name] + "; network trained on seeds 0 and 1 of the same family",
                                    net.n_params)
            plain = runs["plain"]
        else:
            P.reset()
            phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
            rep = P.solve(phi, tol=1e-8, max_iters=50000, raise_on_not_converged=False)
            plain = {"seconds": round(rep["seconds"], 4), "sweeps": rep["iterations"], "residual": rep["residual"]}
        solve = dict(method="plain source iteration", tol=1e-8, **plain)
    P.close()
    del P
    torch.cuda.synchronize()

    mixed = None
    if name == "c5" and prec == 0 and not args.no_secondary:
        # the same sweep in mixed precision: A^{-1} kept in FP32 (half the
        # bytes of the stream that bounds the FP64 sweep), FP64 sums
        t0 = time.perf_counter()
        Pm = Problem.from_workload(ctx, wp, precision=1, schedule=2, cache_inverse=cache)
        ml = sweep_line(Pm, wp, name, 2, 1, args.steps, args.warmup)
        mixed = {"precision": "mixed (A^-1 in FP32, FP64 products and sums; parity bar 1e-5)",
                 "value": ml["value"], "unit": "DOF-dir/s", "ms_per_step": ml["ms_per_step"],
                 "setup_s": round(time.perf_counter() - t0, 2), "roofline": ml["roofline"]}
        note(f"{name} mixed: {ml['ms_per_step']} ms per sweep")
        Pm.close()
        del Pm
        torch.cuda.synchronize()

    secondary = None
    if name == "c5" and not args.no_secondary:
        wp2 = W.c2()
        P2 = Problem.from_workload(ctx, wp2, schedule=1)
        sec = sweep_line(P2, wp2, "c2", 1, 0, args.steps, args.warmup)
        secondary = {"workload": sec["config"]["workload"], "value": sec["value"], "unit": "DOF-dir/s",
                     "ms_per_step": sec["ms_per_step"], "roofline": sec["roofline"]}
        P2.close()
        # and in mixed precision (the persistent kernel with FP32 inverses)
        P2 = Problem.from_workload(ctx, wp2, precision=1)
        s2 = P2.info()["schedule"]
        sm = sweep_line(P2, wp2, "c2", s2, 1, args.steps, args.warmup)
        secondary["mixed"] = {"precision": "mixed (A^-1 in FP32, FP64 products and sums; parity bar 1e-5)",
                              "schedule": "persistent" if s2 == 1 else "levels", "value": sm["value"],
                              "unit": "DOF-dir/s", "ms_per_step": sm["ms_per_step"], "roofline": sm["roofline"]}
        note(f"c2 mixed: {sm['ms_per_step']} ms per sweep")
        P2.close()

    cpu = None
    if not args.no_cpu_baseline:
        if name == "c5":
            cpu = cpu_baseline(wp, block=12, n_dirs_sample=84)
        elif wp.dim == 3:
            cpu = cpu_baseline(wp, block=16, n_dirs_sample=40)
        else:
            cpu = cpu_baseline(wp)

    line = {
        "metric": METRIC,
        "value": main_line["value"],
        "unit": "DOF-dir/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_line["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": main_line["config"],
        "roofline": main_line["roofline"],
        "solve_to_1e-8": solve,
        "learned_vs_plain": learned,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "secondary": secondary,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
