#!/usr/bin/env python3
"""Benchmark of the graph-based S_N transport sweep on one MI355X.

Metric: DOF-direction updates per second of one full lagged sweep (every
level of the combined schedule, the scattering source and the scalar-flux
reduction), E*n*D / t_sweep, with all inputs resident in HBM.  Default
workload: 2D 128x128 Q3 curved mesh (warp 0.3 element widths, 4-element
wavelength, so the sweep graphs have cycles), DG p=3, S8 (40 directions),
sigma_t = 1, c = 0.8, q = 1, vacuum; seeded synthetic inputs.

Also reported: the roofline of the sweep kernel (algorithmic FP64 flops per
launch over its average launch time, HIP events around every launch in a
second timed pass), plain source-iteration time to a 1e-8 residual, the
time to a 1e-8 residual with and without the learned correction on the
two-material c = 0.99 family (training included, reported separately), and
the CPU oracle timed on a sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--workload c2|c1|c3|c4|c5]
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
# HBM bytes per launch of the timed kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes, scaled by a copy kernel of known size (fetch x2.000,
# write x1.000); profiles/sweep_persistent_dpp_c2_128x128_q3_p3_s8.md and
# profiles/sweep_level_inv_c3_32cube_q2_p2_s8.md.  Only valid for the kernel
# build it was measured on: drop an entry when the kernel changes.
MEASURED_TRAFFIC = {("sweep_persistent_dpp<2,3,inv,nt>", "c2", "fp64"): 1.903e9,
                    ("sweep_level_inv<3,2>", "c3", "fp64"): 1.456e8}
DESCRIPTIONS = {
    "c1": "2D 8x8 Q2 curved (warp 0.05), p=1, S4 (12 dirs), sigma_t=1, c=0.5, q=1, vacuum",
    "c2": "2D 128x128 Q3 curved (warp 0.3 h, 4-element wavelength, cyclic sweep graphs), p=3, "
          "S8 (40 dirs), sigma_t=1, c=0.8, q=1, vacuum",
    "c3": "3D 32^3 Q2 curved (warp 0.05), p=2, S8 (80 dirs), checkerboard sigma_t {1,10}, c=0.9, "
          "q=1 in the central 8^3 block, vacuum",
    "c5": "3D 48^3 Q2 curved (warp 0.05), p=2, S12 (168 dirs), random sigma_t {1,100}, c=0.99, "
          "q=1, vacuum",
    "c4": "batch of 64 independent 2D problems (seed 0): m^2 Q2 meshes m in [16,96], p in {1,2,3}, "
          "S4-S12, sigma_t log-uniform [0.1,10], c uniform [0,0.95], q=1, vacuum; one hipGraph "
          "replay per batch sweep, schedule per (dim, p) class chosen by the autotuner",
}


def flops_per_pair(dim: int, p: int) -> float:
    """Algorithmic FP64 flops of one (element, direction) solve: assembly of
    sigma_t M - sum_i Omega_i K_i (2(d+1)n^2), face blocks from the normal
    moments (2d faces x 2d nf^2) with d outflow additions (nf^2) and d inflow
    products (2 nf^2), Gaussian elimination (2/3 n^3) and the two triangular
    sweeps (2 n^2)."""
    n = (p + 1) ** dim
    nf = (p + 1) ** (dim - 1)
    return (2.0 / 3.0) * n ** 3 + 2 * n ** 2 + 2 * (dim + 1) * n ** 2 + 4 * dim * dim * nf ** 2 \
        + 3 * dim * nf ** 2


HBM_PEAK_GBS = 8000.0


def bytes_per_pair_inverse(dim: int, p: int) -> float:
    """Algorithmic HBM bytes of one (element, direction) update when the
    element inverses are cached: the pair's A^{-1} (n^2 doubles), its new
    angular flux (n) and the upwind traces it reads (d inflow faces of nf
    values); the source term (n per element) is counted per element."""
    n = (p + 1) ** dim
    nf = (p + 1) ** (dim - 1)
    return 8.0 * (n * n + n + dim * nf)


def cpu_baseline(wp, n_dirs_sample: int = 4, repeats: int = 1):
    """Time the oracle's sweep on a sample of the directions of the workload."""
    import numpy as np
    from oracle.discretization import Discretization
    from oracle.quadrature import level_symmetric
    from oracle.sweep import build_graphs, sweep
    om, w = level_symmetric(wp.sn_order, wp.dim)
    sel = np.linspace(0, len(w) - 1, min(n_dirs_sample, len(w))).round().astype(int)
    disc = Discretization(wp, omega=om[sel], w=w[sel])
    gs = build_graphs(disc)
    phi = np.zeros((disc.E, disc.n))
    psi = np.zeros((disc.D, disc.E, disc.n))
    t0 = time.perf_counter()
    for _ in range(repeats):
        psi, phi = sweep(disc, gs, phi, psi)
    dt = time.perf_counter() - t0
    threads = 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([1] + [int(i.get("num_threads", 1)) for i in threadpool_info()])
    except Exception:
        pass
    value = disc.E * disc.n * disc.D * repeats / dt
    return {"value": value, "unit": "DOF-dir/s", "cores": threads, "kind": "oracle",
            "sample": f"{repeats} sweep(s) of {len(sel)} of {len(w)} directions (ids {sel.tolist()}) "
                      f"on the full mesh, {dt:.2f} s"}


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
    flops = sum(flops_per_pair(wp.dim, wp.p) * P.E * P.D for wp, P in zip(wps, problems))
    achieved = flops / (ms * 1e-3) / 1e12
    classes = B.classes()
    inv = all(P.info()["cached_inverse"] for P in problems)
    if inv:
        nbytes = sum(bytes_per_pair_inverse(wp.dim, wp.p) * P.E * P.D + 8.0 * P.E * P.n
                     for wp, P in zip(wps, problems))
        gbs = nbytes / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None, "algorithmic_bytes_per_sweep": nbytes,
                "kernel": "whole batch sweep (graph replay: source, fill, class sweeps, scalar flux)"}
    else:
        roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 5), "traffic": None,
                "kernel": "whole batch sweep (graph replay: source, fill, class sweeps, scalar flux)"}
    line = {
        "metric": "DOF-direction updates/s per sweep; time to 1e-8 residual, learned vs plain SI",
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


def learned_vs_plain(nx=16, p=2, sn_order=8, train_seeds=(0, 1, 2, 3), eval_seeds=(100, 101), steps=3000,
                     every=40, stride=3, tol_train=1e-12, verbose=False):
    """Time to a 1e-8 residual with and without the learned correction on
    the two-material c = 0.99 family (the 48^3 S12 configuration's
    materials at nx^3): train on plain-SI pairs (every `stride`-th iteration
    of a solve to tol_train) of train_seeds, evaluate on held-out
    eval_seeds.  Returns a JSON-ready dict."""
    import torch
    import workloads as W
    from paper_1810_11080_amd import Context, Net, Problem
    from paper_1810_11080_amd import learn as L

    def note(msg):
        if verbose:
            print(msg, file=sys.stderr, flush=True)

    ctx = Context(device=0)
    t0 = time.perf_counter()
    Xs, Ts = [], []
    for seed in train_seeds:
        P = Problem.from_workload(ctx, W.c5_reduced(seed=seed, nx=nx, p=p, sn_order=sn_order))
        kept, star, its = L.plain_trajectory(P, tol=tol_train, max_iters=50000, sample=lambda l: l % stride == 0,
                                             progress=note if verbose else None)
        X, T = L.make_pairs(P, kept, star)
        Xs.append(X)
        Ts.append(T)
        note(f"training seed {seed}: {its} plain sweeps, {len(kept)} pairs, {time.perf_counter() - t0:.1f} s")
        del kept, P
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    net = Net(ctx, widths=(16, 32, 32), seed=0)
    t0 = time.perf_counter()
    losses = L.train(net, (nx, nx, nx), X, T, steps=steps, batch=8, lr=2e-3, lr_final=1e-4,
                     log_every=500 if verbose else 0)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    runs = []
    for seed in eval_seeds:
        P = Problem.from_workload(ctx, W.c5_reduced(seed=seed, nx=nx, p=p, sn_order=sn_order))
        row = {"seed": seed}
        for name, pre in (("plain", None), ("learned", net)):
            P.reset()
            phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
            rep = P.solve(phi, tol=1e-8, max_iters=50000, precond=pre, precond_every=every)
            row[name] = {"seconds": round(rep["seconds"], 4), "sweeps": rep["iterations"]}
            note(f"eval seed {seed} {name}: {row[name]}")
            if pre is not None:
                row[name].update(corrections=rep["n_corrected"], rejected=rep["n_rejected"])
        runs.append(row)
    plain = sum(r["plain"]["seconds"] for r in runs)
    learned = sum(r["learned"]["seconds"] for r in runs)
    saved = (plain - learned) / len(runs)
    return {"workload": f"3D {nx}^3 Q2 (warp 0.05), p={p}, S{sn_order}, sigma_t in {{1,100}} (random, 50/50), "
                        f"c=0.99, q=1, vacuum; trained on seeds {list(train_seeds)}, evaluated on "
                        f"{list(eval_seeds)}",
            "tol": 1e-8, "precond_every": every, "params": net.n_params,
            "time_plain_s": round(plain / len(runs), 4), "time_learned_s": round(learned / len(runs), 4),
            "speedup": round(plain / learned, 3), "runs": runs,
            "training": {"pairs": int(X.shape[0]), "data_s": round(data_s, 2), "train_s": round(train_s, 2),
                         "steps": steps, "loss_first": float(losses[:10].mean()),
                         "loss_last": float(losses[-100:].mean()),
                         "break_even_solves": round((data_s + train_s) / saved, 1) if saved > 0 else None}}


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
    ap.add_argument("--workload", default="c2", choices=sorted(DESCRIPTIONS),
                    help="c2 (default): the single-problem benchmark; c4: the 64-problem batch")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--schedule", default="auto", choices=["auto", "persistent", "levels"])
    ap.add_argument("--cache-inverse", default="auto", choices=["auto", "on", "off"],
                    help="keep each pair's A^{-1} on the device (factored once at setup)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain comparison")
    ap.add_argument("--learned-only", choices=["c5"], default=None,
                    help="only the learned-vs-plain comparison at the full 48^3 S12 size (minutes)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a copy kernel of known size (HBM counter calibration)")
    ap.add_argument("--weighting-study", action="store_true",
                    help="only the unity / face / sigma-inverse-face weighting comparison")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(directions would be sharded across GPUs with one scalar-flux all-reduce "
              "per iteration; not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
    if args.learned_only == "c5":
        res = learned_vs_plain(nx=48, p=2, sn_order=12, train_seeds=(0, 1), eval_seeds=(100,), steps=2000,
                               every=40, stride=10, tol_train=1e-10, verbose=True)
        print(json.dumps({"learned_vs_plain": res}))
        return
    if args.workload == "c4":
        bench_batch(args)
        return
    wp = W.CONFIGS[args.workload]()
    prec = 0 if args.precision == "fp64" else 1
    ctx = Context(device=0)
    t0 = time.perf_counter()
    sched = {"auto": 0, "persistent": 1, "levels": 2}[args.schedule]
    if sched == 0:   # same rule as the library's automatic choice
        sched = 1 if (wp.dim == 2 and wp.p != 2 and prec == 0) else 2
    cache = {"auto": 0, "on": 1, "off": 2}[args.cache_inverse]
    P = Problem.from_workload(ctx, wp, precision=prec, schedule=sched, cache_inverse=cache)
    setup_s = time.perf_counter() - t0
    info = P.info()
    E, n, D = P.E, P.n, P.D
    phi = torch.zeros(E * n, dtype=torch.float64, device="cuda")
    out = torch.empty_like(phi)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        P.sweep(phi, out)
        phi, out = out, phi
    torch.cuda.synchronize()
    # timed pass: whole sweeps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        P.sweep(phi, out)
        phi, out = out, phi
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    dof_dir = E * n * D
    value = dof_dir / (ms_per_step * 1e-3)

    # second timed pass: HIP events around every level-sweep launch
    P.profile_enable(True)
    for _ in range(args.steps):
        P.sweep(phi, out)
        phi, out = out, phi
    launches, kernel_ms = P.profile_read()
    P.profile_enable(False)
    P.synchronize()
    launches_per_sweep = launches / args.steps
    avg_launch_ms = kernel_ms / launches
    flops_sweep = flops_per_pair(wp.dim, wp.p) * E * D
    flops_per_launch = flops_sweep / launches_per_sweep
    achieved = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    inv = bool(info["cached_inverse"])
    if sched == 1:
        if wp.dim == 2 and wp.p != 2:
            nt = ",nt" if inv and info["tile"] > 0 else ""
            kname = f"sweep_persistent_dpp<{wp.dim},{wp.p}{',inv' if inv else ''}{nt}>"
        elif inv:
            kname = f"sweep_persistent_lds2d<{wp.p}>" if wp.dim == 2 else f"sweep_persistent_inv<{wp.dim},{wp.p}>"
        else:
            kname = f"sweep_persistent_fp64<{wp.dim},{wp.p}>"
    else:
        kname = f"sweep_level_inv<{wp.dim},{wp.p}>" if inv else f"sweep_level_fp64<{wp.dim},{wp.p}>"
    if inv:
        # cached inverses: the sweep streams A^{-1}; HBM bound
        bytes_sweep = bytes_per_pair_inverse(wp.dim, wp.p) * E * D + 8.0 * E * n
        gbs = bytes_sweep / launches_per_sweep / (avg_launch_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 5),
                    "traffic": MEASURED_TRAFFIC.get((kname, args.workload, args.precision)),
                    "kernel": kname, "algorithmic_bytes_per_sweep": bytes_sweep,
                    "avg_launch_us": round(avg_launch_ms * 1e3, 3), "launches_per_sweep": launches_per_sweep,
                    "kernel_share_of_step": round(kernel_ms / args.steps / ms_per_step, 4),
                    "fp64_alu_view_tflops": round(achieved, 4)}
    else:
        roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_VECTOR_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 5),
                    "traffic": MEASURED_TRAFFIC.get((kname, args.workload, args.precision)),
                    "kernel": kname,
                    "avg_launch_us": round(avg_launch_ms * 1e3, 3),
                    "launches_per_sweep": launches_per_sweep,
                    "kernel_share_of_step": round(kernel_ms / args.steps / ms_per_step, 4)}

    solve = None
    if not args.no_solve:
        P.reset()
        phi.zero_()
        rep = P.solve(phi, tol=1e-8, max_iters=2000, check_every=1, raise_on_not_converged=False)
        solve = {"method": "plain source iteration", "tol": 1e-8, "iterations": rep["iterations"],
                 "seconds": round(rep["seconds"], 4), "residual": rep["residual"]}

    learned = None
    if not args.no_learned and args.workload == "c2":
        learned = learned_vs_plain()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wp, n_dirs_sample=40 if args.workload in ("c1", "c2") else 4)

    line = {
        "metric": "DOF-direction updates/s per sweep; time to 1e-8 residual, learned vs plain SI",
        "value": value,
        "unit": "DOF-dir/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS[args.workload], "elements": E, "dofs_per_element": n,
                   "directions": D, "levels": info["n_levels_total"],
                   "lagged_edges": info["n_removed_total"], "kink_face_dirs": info["n_kink_faces_total"],
                   "setup_s": round(setup_s, 2), "precision": args.precision,
                   "cached_inverse": inv,
                   "schedule": "persistent" if sched == 1 else "levels"},
        "roofline": roofline,
        "solve_to_1e-8": solve,
        "learned_vs_plain": learned,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
