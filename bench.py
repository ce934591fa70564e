"""Benchmark: time steps/s of the hot path on one MI355X.

Workload (default): the mixed-precision plain method at scale -- channel with
one seeded circular obstacle (seed 0), Re = 100, macro mesh refined to level 7
(1.38M cells, ~1.38M nodes, ~4.1M DoFs), dt = 0.005, FP32 smoother, transfers
and Krylov vectors with FP64 Newton residual, update, coarse solve and
Gram-Schmidt dots.  W untimed steps from rest, then K timed steps.

Prints one JSON line (see the field list at the bottom).  `roofline` is
computed from per-kernel HIP-event timings recorded by the library on its
stream over the timed region; `cpu_baseline` times the FP64 oracle on a
bounded sample (one Newton-direct step on a coarser level of the same
geometry, scaled to the level-7 step by the DoF ratio).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time steps/s, DNN-MG vs full-depth GMG, 1 GPU at fixed velocity L2 err"
HBM_PEAK_GBS = 8000.0


def kernel_bytes(ctx, key, level):
    """Algorithmic bytes of one launch of the kernel `key` on `level`
    (FP32 operator/vectors, 4-byte indices; each array counted once)."""
    n, c, p = ctx.level_info(level)
    st = ctx.level_stats(level)
    qb, xe = st["q_blocks"], st["x_entries"]
    f = 4
    if key == "spmv":          # y = J x
        return 9 * qb * f + xe * f + (qb + xe) * 4 + 3 * n * f + 3 * n * f
    if key == "residual_spmv":  # y = b - J x
        return 9 * qb * f + xe * f + (qb + xe) * 4 + 3 * 3 * n * f
    if key == "vanka_apply":   # inverse blocks, cell nodes, r gather, delta write
        return 144 * c * f + 16 * c + 3 * n * f + 12 * c * f
    if key == "vanka_update":  # node->cell list, delta, x read/write
        return 4 * c * 4 + 4 * n + 12 * c * f + 2 * 3 * n * f
    return None


def cpu_baseline(seed: int, level: int, fine_level: int, dt: float):
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import fem, mesh, solver
    from synthetic import channel_obstacle
    macro = channel_obstacle(seed)
    lev = mesh.hierarchy(macro, level)
    L = lev[level]
    prob = fem.Problem(nu=macro.nu, dt=dt)
    x = np.zeros(3 * L.n_nodes)
    x = solver.newton_step(L, prob, x, dt, tol=1e-10)      # untimed first step
    t0 = time.perf_counter()
    x = solver.newton_step(L, prob, x, 2 * dt, tol=1e-10)
    sec = time.perf_counter() - t0
    cells_fine = L.n_cells * 4 ** (fine_level - level)
    scale = cells_fine / L.n_cells
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": 1.0 / (sec * scale), "unit": "time steps/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"one FP64 Newton step with direct sparse solves at level {level} "
                       f"({3 * L.n_nodes} DoFs, {sec:.2f} s), scaled by the cell ratio "
                       f"{scale:.0f} to the level-{fine_level} step")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--level", type=int, default=7)
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-level", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_2106_07687_amd as P
    from synthetic import channel_obstacle

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    macro = channel_obstacle(args.seed)
    ctx = P.Context(precision=1, nu=macro.nu, stream=stream.cuda_stream)
    t0 = time.perf_counter()
    ctx.setup_mesh(macro, args.level)
    setup_s = time.perf_counter() - t0
    n_nodes, n_cells, _ = ctx.level_info(args.level)
    st = ctx.state(args.level)
    print(f"[bench] setup level {args.level}: {n_nodes} nodes, {n_cells} cells, "
          f"{setup_s:.1f} s", file=sys.stderr, flush=True)
    for k in range(args.warmup):
        info = ctx.step(st, args.dt)
        print(f"[bench] warmup step {k}: {info}", file=sys.stderr, flush=True)
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        stats.append(ctx.step(st, args.dt))
    stream.synchronize()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    prof = ctx.profile_report()
    ctx.profile_enable(False)
    for k, s in enumerate(stats):
        print(f"[bench] step {k}: {s}", file=sys.stderr, flush=True)

    # dominant kernel on the finest level with a traffic model
    best = None
    for key, (cnt, ms) in prof.items():
        name, lv = key.split("@L")
        if int(lv) != args.level:
            continue
        b = kernel_bytes(ctx, name, args.level)
        if b is None:
            continue
        if best is None or ms > best[2]:
            best = (name, cnt, ms, b)
    roof = None
    if best:
        name, cnt, ms, b = best
        avg_s = ms / cnt / 1e3
        ach = b / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": f"{name}@L{args.level}", "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": None, "avg_us": round(avg_s * 1e6, 2), "launches": cnt,
                "bytes_per_launch": b}
    for key in sorted(prof, key=lambda k: -prof[k][1])[:12]:
        cnt, ms = prof[key]
        print(f"[bench] kernel {key}: {cnt} launches, {ms:.2f} ms total, "
              f"{1e3 * ms / cnt:.1f} us avg", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.seed, args.cpu_level, args.level, args.dt)
    ms_step = 1e3 * sec / args.steps
    out = {
        "metric": METRIC,
        "value": round(args.steps / sec, 4),
        "unit": "time steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"plain full-depth GMG, channel+obstacle seed {args.seed}, "
                               f"level {args.level}, Re 100, dt {args.dt}, mixed precision",
                   "level": args.level, "nodes": n_nodes, "dofs": 3 * n_nodes,
                   "newton_iters": sum(s["newton_iters"] for s in stats),
                   "gmres_iters": sum(s["gmres_iters"] for s in stats),
                   "dof_updates_per_s": round(3 * n_nodes * args.steps / sec, 1)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
