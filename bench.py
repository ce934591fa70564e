"""Benchmark: time steps/s of DNN-MG against full-depth GMG on one MI355X.

Workload: channel with one seeded circular obstacle (seed 0), Re = 100,
dt = 0.005, mixed precision (FP32 smoother, transfers and Krylov vectors;
FP64 Newton residual, update, coarse solve and Gram-Schmidt dots).
  * full-depth GMG: Newton-GMRES-multigrid on level 7 (1.38M cells, ~4.1M
    DoFs), W untimed steps from rest, then K timed steps;
  * DNN-MG: Newton-GMRES-multigrid on level 5 plus the patch GRU (hidden 128,
    2 layers, BF16 MFMA) correcting level 7 (Algorithm 1), W + K steps;
`value` is the DNN-MG rate; the GMG rate, the speed-up and the velocity
errors of DNN-MG and of the plain level-5 method against the level-7
solution are reported in `config`.  `train` times BPTT iterations at the
training batch shape (8192 sequences x 32 steps).

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


def run_batch(P, args, log):
    """Batched plain solves: seeded multi-obstacle channels (seeds 100, 101, ...),
    each at its own Re and depth (4-7), all advanced together."""
    import torch

    from synthetic import channel_obstacles
    macros = [channel_obstacles(s) for s in range(100, 100 + args.batch_sims)]
    t0 = time.perf_counter()
    batch = P.Batch([(m, m.nu, m.info["depth"]) for m in macros], precision=1)
    setup_s = time.perf_counter() - t0
    groups = [batch.group_info(g) for g in range(batch.n_groups())]
    log(f"batch: {args.batch_sims} simulations in {len(groups)} depth groups {groups}, "
        f"setup {setup_s:.1f} s")
    for k in range(args.batch_warmup):
        log(f"batch warmup {k}: {batch.step(args.dt)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [batch.step(args.dt) for _ in range(args.batch_steps)]
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    for k, st in enumerate(stats):
        log(f"batch step {k}: {st}")
    dofs = sum(3 * g["n_nodes"] for g in groups)
    out = {"simulations": args.batch_sims, "seeds": f"100..{99 + args.batch_sims}",
           "groups": [dict(g, newton_iters=sum(st[i]["newton_iters"] for st in stats),
                           gmres_iters=sum(st[i]["gmres_iters"] for st in stats))
                      for i, g in enumerate(groups)],
           "dofs": dofs, "steps": args.batch_steps, "warmup": args.batch_warmup,
           "steps_per_s": round(args.batch_steps / sec, 4),
           "sim_steps_per_s": round(args.batch_sims * args.batch_steps / sec, 3),
           "dof_updates_per_s": round(dofs * args.batch_steps / sec, 1),
           "setup_s": round(setup_s, 2), "precision": "mixed"}
    batch.close()
    return out


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


def run_steps(ctx, st, steps, dt, net=None):
    """`steps` time steps (plain, or DNN-MG: coarse step + correction)."""
    stats = []
    for _ in range(steps):
        stats.append(ctx.step(st, dt))
        if net is not None:
            net.correct(st, dt)
    return stats


def fine_state(ctx, xl, level, fine_level, corr=None):
    """P^m x^L on the fine level, with the network's velocity correction added."""
    x = xl
    for l in range(level + 1, fine_level + 1):
        x = ctx.prolong(l, x)
    if corr is not None:
        x = x.reshape(-1, 3).copy()
        x[:, :2] += corr
        x = x.reshape(-1)
    return x


def velocity_error(ctx, xl, level, fine_level, x_fine, corr=None):
    """Relative l2 error of the fine-level velocity (P^m v^L [+ d]) against
    the fine solution."""
    import numpy as np
    x = xl
    for l in range(level + 1, fine_level + 1):
        x = ctx.prolong(l, x)
    v = x.reshape(-1, 3)[:, :2]
    if corr is not None:
        v = v + corr
    ref = x_fine.reshape(-1, 3)[:, :2]
    return float(np.linalg.norm(v - ref) / np.linalg.norm(ref))


# the kernels that run these keys on level 7 of the benchmark mesh (the
# autotuner takes the cell-ordered update there)
KERNEL_OF = {"spmv": "k_spmv", "residual_spmv": "k_spmv", "vanka_apply": "k_vanka_apply",
             "vanka_update": "k_vanka_update_ordered"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_level7_kernels.md")


def kernel_sha1(kernel):
    """SHA-1 of a kernel's source text in csrc/kernels.h: its definition plus
    the definitions of the device functions it calls (transitively)."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_2106_07687_amd", "csrc", "kernels.h")).read()

    def definition(name, kind):
        m = re.search(kind + r"[^;{]*?\b" + name + r"\(", src)
        if not m:
            return None
        i = src.index("{", m.end())
        depth = 0
        for j in range(i, len(src)):
            depth += {"{": 1, "}": -1}.get(src[j], 0)
            if depth == 0:
                return src[m.start():j + 1]
        return None

    text = definition(kernel, "__global__")
    if text is None:
        return None
    parts, seen, todo = [text], {kernel}, [text]
    while todo:
        body = todo.pop()
        for callee in re.findall(r"\b([a-z_0-9]+_(?:item|row))\(", body):
            if callee not in seen:
                seen.add(callee)
                d = definition(callee, "__device__")
                if d:
                    parts.append(d)
                    todo.append(d)
    return hashlib.sha1("\n".join(parts).encode()).hexdigest()


def measured_traffic(name, level):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated against a copy kernel), or None when
    the kernel's source has changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE) or name not in KERNEL_OF:
        return None
    sha = kernel_sha1(KERNEL_OF[name])
    for line in open(TRAFFIC_FILE):
        f = line.split()
        if len(f) == 5 and f[0] == "traffic" and f[1] == name and f[2] == f"L{level}":
            if f[3] == f"sha1={sha}":
                return int(f[4].split("=")[1])
    return None


def roofline_from(prof, ctx, level, kernels_with_bytes, log=None):
    rows = []
    for key, (cnt, ms) in prof.items():
        name, lv = key.split("@L")
        if int(lv) != level or name not in kernels_with_bytes:
            continue
        b = kernel_bytes(ctx, name, level)
        if b is None:
            continue
        avg_s = ms / cnt / 1e3
        rows.append((ms, name, cnt, avg_s, b))
        if log:
            log(f"roofline {name}@L{level}: {b / 1e6:.1f} MB/launch algorithmic, {avg_s * 1e6:.1f} us, "
                f"{b / avg_s / 1e9:.0f} GB/s, measured traffic {measured_traffic(name, level)}")
    if not rows:
        return None
    _, name, cnt, avg_s, b = max(rows)
    ach = b / avg_s / 1e9
    return {"bound": "hbm", "kernel": f"{name}@L{level}", "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(name, level), "avg_us": round(avg_s * 1e6, 2),
            "launches": cnt, "bytes_per_launch": b}


def teacher_data(ctx, net, xF, L, dt, n0=1, t0=0.0):
    """Teacher-forced coarse steps n = n0 .. len(xF) - 1 (xF[k] is the fine
    state at t0 + k dt; the coarse right-hand side is restricted from the
    fine velocity of the previous step): raw network inputs (T, B, I) and
    targets d* = v^F_n - P^m v^L_n (T, B, O).  Inputs and targets do not
    depend on the network's weights, only on its patches."""
    import numpy as np
    nL = ctx.level_info(L)[0]
    net.set_weights(None, mu=np.zeros(net.n_stats), sigma=np.ones(net.n_stats), out_scale=np.ones(2))
    sl = ctx.state(L)
    Xr, Dr = [], []
    for n in range(n0, len(xF)):
        sl.set(xF[n - 1][:3 * nL], t0 + (n - 1) * dt)
        net.rhs_from_fine(sl, xF[n - 1], dt)
        ctx.step(sl, dt)
        Xr.append(net.correct(sl, dt, debug=True)["inputs"])
        Dr.append(net.targets(sl, xF[n]))
    sl.close()
    return np.stack(Xr), np.stack(Dr)


def standardisation(net, Xr, Dr):
    """Per-channel (mu, sigma) of the raw inputs and the two output scales,
    and their per-column expansions."""
    import numpy as np
    S2 = net.n_out // 2
    nch = (net.n_in - net.n_stats) // (S2 - 1)        # nodal channels (6 block, 5 cell)
    nft = net.n_stats - nch
    mu = np.array([Xr[..., c * S2:(c + 1) * S2].mean() for c in range(nch)] +
                  [Xr[..., nch * S2 + k].mean() for k in range(nft)])
    sg = np.array([Xr[..., c * S2:(c + 1) * S2].std() for c in range(nch)] +
                  [Xr[..., nch * S2 + k].std() for k in range(nft)])
    sg = np.where(sg > 1e-30, sg, 1.0)
    osc = np.array([Dr[..., :S2].std(), Dr[..., S2:].std()])
    osc = np.where(osc > 1e-30, osc, 1.0)
    mu_f = np.concatenate([np.repeat(mu[:nch], S2), mu[nch:]]).astype(np.float32)
    sg_f = np.concatenate([np.repeat(sg[:nch], S2), sg[nch:]]).astype(np.float32)
    os_f = np.concatenate([np.repeat(osc[0], S2), np.repeat(osc[1], S2)]).astype(np.float32)
    return (mu, sg, osc), (mu_f, sg_f, os_f)


class Fitter:
    """BPTT + Adam on device-resident sequences; keeps the wall time of the
    training iterations alone (each call returns its loss: synchronous)."""

    def __init__(self, net, X, D, ckpt=8):
        self.net, self.X, self.D = net, X, D
        self.ckpt = min(ckpt, X.shape[0])
        self.iters, self.sec = 0, 0.0

    def __call__(self, n_it, lr):
        import torch
        loss = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T, B = self.X.shape[0], self.X.shape[1]
        for it in range(n_it):
            loss = self.net.train_step_dev(self.X.data_ptr(), self.D.data_ptr(), T, B,
                                           lr=lr if it < 0.75 * n_it else 0.3 * lr, ckpt=self.ckpt)
        self.sec += time.perf_counter() - t0
        self.iters += n_it
        return loss


def train_dnnmg(ctx, net, xF, L, dt, iters, dagger, seed, log):
    """Trains the patch network on the GPU (untimed in the step benchmark):
    teacher-forced inputs and targets, BPTT with Adam, then DAgger rounds that
    add the states of free DNN-MG runs."""
    import numpy as np
    import torch

    from synthetic import gru_weights
    N = len(xF) - 1
    Xr, Dr = teacher_data(ctx, net, xF, L, dt)
    (mu, sg, osc), (mu_f, sg_f, os_f) = standardisation(net, Xr, Dr)
    w0 = gru_weights(net.n_in, net.hidden, net.layers, net.n_out, seed=seed, scale=0.5)
    net.set_weights(w0, mu=mu, sigma=sg, out_scale=osc)
    X = torch.from_numpy((Xr - mu_f) / sg_f).cuda()
    D = torch.from_numpy(Dr / os_f).cuda()
    del Xr, Dr
    fit = Fitter(net, X, D)
    first = net.train_step_dev(X.data_ptr(), D.data_ptr(), N, X.shape[1], lr=2e-3, ckpt=fit.ckpt)
    loss = fit(iters, 2e-3)
    log(f"net training (teacher forcing): loss {first:.1f} -> {loss:.1f}, {X.shape[1]} sequences")
    for rnd in range(dagger):
        st = ctx.state(L)
        net.reset(st)
        Xc, Dc = [], []
        for n in range(1, N + 1):
            ctx.step(st, dt)
            Xc.append(net.correct(st, dt, debug=True)["inputs"])
            Dc.append(net.targets(st, xF[n]))
        st.close()
        fit.X = torch.cat([fit.X, torch.from_numpy(np.stack(Xc)).cuda()], dim=1).contiguous()
        fit.D = torch.cat([fit.D, torch.from_numpy(np.stack(Dc)).cuda()], dim=1).contiguous()
        loss = fit(iters // 2, 1e-3)
        log(f"net training (DAgger round {rnd}): loss {loss:.1f}, {fit.X.shape[1]} sequences")
    del fit
    torch.cuda.empty_cache()
    return {"sequences_per_round": net.n_patches, "steps": N, "rounds": 1 + dagger,
            "final_loss": round(float(loss), 3)}


TABLE1_SHAPES = ((32, 1), (64, 1), (32, 2), (64, 2), (32, 3), (64, 3))


def run_table1(P, args, log):
    """The network-size sweep of Table 1 / Table 2 and the lift comparison of
    Sec. 3.3 on one MI355X: cell patches (one level-L element, I = 51, O = 18)
    correcting level F = L + 1, the six GRU shapes.  A fine run MG(F) from
    rest to t_end gives the reference; each network trains on teacher-forced
    32-step sequences from [t_train, t_start); MG(L) and every DNN-MG run
    restart from the fine state at t_start (injected to level L) and run to
    t_end.  Per run: steps/s, velocity error and the lift's period and phase
    offset against MG(F) over the last time unit (dnnmg_oscillation)."""
    import numpy as np
    import torch

    from synthetic import channel_obstacle, gru_weights
    macro = channel_obstacle(args.seed)
    F = args.t1_level
    L = F - 1
    dt = args.t1_dt
    n_end = int(round(args.t1_end / dt))
    n_start = int(round(args.t1_start / dt))
    n_train = int(round(args.t1_train_from / dt))
    seq = 32
    n_train = n_start - (n_start - n_train) // seq * seq           # whole sequences
    w0 = n_end - int(round(1.0 / dt))                              # analysis window [t_end - 1, t_end]
    ctx = P.Context(precision=1, nu=macro.nu, jacobian_reuse=args.jacobian_reuse)
    ctx.setup_mesh(macro, F)
    nL = ctx.level_info(L)[0]

    def lift_of(st):
        return float(st.functionals(1)[2][0])

    sf = ctx.state(F)
    xF, liftF = [sf.get()[0]], [0.0]
    fine_sec = 0.0
    for _ in range(n_end):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(sf, dt)
        torch.cuda.synchronize()
        fine_sec += time.perf_counter() - t0
        xF.append(sf.get()[0])
        liftF.append(lift_of(sf))
    sf.close()
    osc_F = P.oscillation(liftF[w0:], w0 * dt, dt)

    def restart(net):
        st = ctx.state(L)
        st.set(xF[n_start][:3 * nL], n_start * dt)
        if net is not None:
            net.reset(st)
            net.rhs_from_fine(st, xF[n_start], dt)
        return st

    def coarse_run(net=None):
        """Restart at t_start from the fine state: a timed pass (steps and
        corrections only), then a pass that also reads the states back; (steps/s,
        mean velocity error over the window, lift oscillation)."""
        st = restart(net)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_steps(ctx, st, n_end - n_start, dt, net)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        st.close()
        st = restart(net)
        lift, err, newton = [], [], []
        builds = fallbacks = 0
        for n in range(n_start + 1, n_end + 1):
            info = ctx.step(st, dt)
            newton.append(info["newton_iters"])
            builds += info["jacobian_builds"]
            fallbacks += info["fallback"]
            corr = net.correct(st, dt, debug=True)["correction"] if net is not None else None
            xl = st.get()[0]
            if n >= w0:
                err.append(velocity_error(ctx, xl, L, F, xF[n], corr))
                lift.append(float(ctx.functionals(F, fine_state(ctx, xl, L, F, corr), 1)[2][0]))
        st.close()
        stats = {"newton_iters": int(sum(newton)), "jacobian_builds": builds, "fallbacks": fallbacks,
                 "newton_first10_median": float(np.median(newton[:10]))}
        return (n_end - n_start) / sec, float(np.mean(err)), P.oscillation(lift, w0 * dt, dt), stats

    def phase(osc):
        """(period, first-maximum offset against MG(F) in periods of MG(F))."""
        off = (osc[0] - osc_F[0]) / osc_F[1]
        return round(osc[1], 5), round(float(off - np.round(off)), 4)

    sps_L, err_L, osc_L, st_L = coarse_run()
    # switch-off (Sec. 3.3): a DNN-MG step whose Newton iteration needs more than
    # twice the plain coarse method's median count over its first 10 steps is
    # redone with the plain right-hand side
    n_off = max(1, int(round(2 * st_L["newton_first10_median"])))
    ctx.set_params(switch_off_newton=n_off)
    out = {"coarse_level": L, "fine_level": F, "dt": dt, "t_train": [n_train * dt, n_start * dt],
           "t_run": [n_start * dt, n_end * dt], "window": [w0 * dt, n_end * dt],
           "coarse_dofs": 3 * nL, "fine_dofs": 3 * ctx.level_info(F)[0],
           "mg_fine": {"steps_per_s": round(n_end / fine_sec, 2), "lift_period": round(osc_F[1], 5)},
           "mg_coarse": {"steps_per_s": round(sps_L, 2), "vel_err": round(err_L, 6),
                         "lift_period": phase(osc_L)[0], "lift_phase_offset": phase(osc_L)[1],
                         "newton_iters": st_L["newton_iters"], "jacobian_builds": st_L["jacobian_builds"]},
           "switch_off_newton": n_off,
           "nets": []}
    log(f"table1 MG(F): {out['mg_fine']}; MG(L): {out['mg_coarse']}")
    probe = P.Net(ctx, L, 1, 32, 1, patch="cell")
    Xr, Dr = teacher_data(ctx, probe, xF[n_train - 1:n_start + 1], L, dt, t0=(n_train - 1) * dt)
    probe.close()
    nseq = Xr.shape[0] // seq
    Xr = Xr[:nseq * seq].reshape(nseq, seq, *Xr.shape[1:]).transpose(1, 0, 2, 3).reshape(seq, -1, Xr.shape[2])
    Dr = Dr[:nseq * seq].reshape(nseq, seq, *Dr.shape[1:]).transpose(1, 0, 2, 3).reshape(seq, -1, Dr.shape[2])
    for H, layers in TABLE1_SHAPES:
        net = P.Net(ctx, L, 1, H, layers, patch="cell")
        (mu, sg, osc), (mu_f, sg_f, os_f) = standardisation(net, Xr, Dr)
        net.set_weights(gru_weights(net.n_in, H, layers, net.n_out, seed=args.seed, scale=0.5),
                        mu=mu, sigma=sg, out_scale=osc)
        X = torch.from_numpy(np.ascontiguousarray((Xr - mu_f) / sg_f)).cuda()
        D = torch.from_numpy(np.ascontiguousarray(Dr / os_f)).cuda()
        fit = Fitter(net, X, D)
        loss = fit(args.t1_iters, 2e-3)
        bptt_ms = 1e3 * fit.sec / fit.iters
        del fit, X, D
        sps, err, osc_d, st_d = coarse_run(net)
        per, off = phase(osc_d)
        row = {"hidden": H, "layers": layers, "params": net.n_params, "n_in": net.n_in, "n_out": net.n_out,
               "sequences": Xr.shape[1], "seq": seq, "bptt_iters": args.t1_iters,
               "bptt_ms_per_iter": round(bptt_ms, 3), "train_sec": round(bptt_ms * args.t1_iters / 1e3, 2),
               "final_loss": round(float(loss), 3),
               "steps_per_s": round(sps, 2), "vel_err": round(err, 6), "lift_period": per,
               "lift_phase_offset": off, "newton_iters": st_d["newton_iters"],
               "jacobian_builds": st_d["jacobian_builds"], "fallbacks": st_d["fallbacks"]}
        log(f"table1 {H}x{layers}: {row}")
        out["nets"].append(row)
        net.close()
        torch.cuda.empty_cache()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--level", type=int, default=7)
    ap.add_argument("--coarse-level", type=int, default=5)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--layers", type=int, default=2)
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-level", type=int, default=4)
    ap.add_argument("--train-iters", type=int, default=3)
    ap.add_argument("--train-seq", type=int, default=32)
    ap.add_argument("--train-batch", type=int, default=8192)
    ap.add_argument("--train-net", type=int, default=1,
                    help="train the patch network on the GPU before the DNN-MG run (untimed)")
    ap.add_argument("--train-net-iters", type=int, default=150)
    ap.add_argument("--dagger", type=int, default=2)
    ap.add_argument("--profile", choices=("roofline", "all"), default="roofline",
                    help="roofline: HIP events only around the fine-level GMG kernels and "
                         "the network kernels; all: every kernel of every level, launched "
                         "directly (no graphs; events add launch overhead to the timings)")
    ap.add_argument("--newton-predictor", type=int, default=1, choices=(0, 1),
                    help="1: Newton starts from the linear extrapolation of the last two states")
    ap.add_argument("--table1", type=int, default=1, choices=(0, 1),
                    help="network-size sweep (Table 1 shapes on cell patches, untimed leg)")
    ap.add_argument("--t1-level", type=int, default=3)
    ap.add_argument("--t1-dt", type=float, default=0.01)
    ap.add_argument("--t1-train-from", type=float, default=4.0)
    ap.add_argument("--t1-start", type=float, default=7.0)
    ap.add_argument("--t1-end", type=float, default=10.0)
    ap.add_argument("--t1-iters", type=int, default=600)
    ap.add_argument("--jacobian-reuse", type=int, default=1, choices=(0, 1),
                    help="keep Newton's Jacobians across iterations and steps while the "
                         "residual contracts by 0.1 or better (0: rebuild every step)")
    ap.add_argument("--nu-coarse", type=int, default=0,
                    help="full-depth GMG leg: sweeps before and after on the V-cycle levels below the "
                         "one GMRES works on (0: the same V(2,2) on every level)")
    ap.add_argument("--dnnmg-sweeps", default="2,1,1",
                    help="pre,post,coarse sweeps of the V-cycles of the DNN-MG leg's level-5 solves "
                         "(measured on level 5: V(2,1) with V(1,1) below is the fastest schedule; the "
                         "GMG leg keeps V(2,2) throughout)")
    ap.add_argument("--direct-level", type=int, default=1, choices=(0, 1, 2),
                    help="level of the direct (FP64 dense inverse) solve at the bottom of every V-cycle, "
                         "both legs (level 1: 1,140 unknowns, one 10 MB mat-vec instead of level-1 "
                         "sweeps and the level-0 solve)")
    ap.add_argument("--smoother", type=int, default=0, choices=(0, 1),
                    help="0: additive cell-Vanka, 1: coloured multiplicative cell-Vanka")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel directly instead of replaying captured graphs")
    ap.add_argument("--batch-sims", type=int, default=64,
                    help="batched plain solves: simulations (0 skips the leg)")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--batch-warmup", type=int, default=1)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="device copy of this many MiB before the run (calibrates "
                         "hardware traffic counters against a known byte count)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2106_07687_amd as P
    from synthetic import channel_obstacle, gru_weights

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.calib_copy_mb > 0:
        src = torch.ones(args.calib_copy_mb * (1 << 18), device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    macro = channel_obstacle(args.seed)
    ctx = P.Context(precision=1, nu=macro.nu, stream=stream.cuda_stream,
                    use_graphs=0 if args.no_graphs else 1, newton_predictor=args.newton_predictor,
                    jacobian_reuse=args.jacobian_reuse, smoother=args.smoother, nu_coarse=args.nu_coarse,
                    coarse_level=args.direct_level)
    F = args.level
    if args.profile == "all":
        gmg_keys = dnn_keys = None
    else:
        gmg_keys = [f"{k}@L{F}" for k in ("spmv", "residual_spmv", "vanka_apply", "vanka_update",
                                          "assemble", "vanka_factor", "residual", "gs_dots")]
        dnn_keys = [f"{k}{l}@L{F}" for l in range(args.layers)
                    for k in ("gru_gemm_in", "gru_step")]
        dnn_keys += [f"{k}@L{F}" for k in ("gru_head", "dnnmg_rhs", "dnnmg_prolong",
                                           "patch_gather", "patch_scatter")]
    t0 = time.perf_counter()
    ctx.setup_mesh(macro, args.level)
    setup_s = time.perf_counter() - t0
    nF, cF, _ = ctx.level_info(args.level)
    nL = ctx.level_info(args.coarse_level)[0]
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    log(f"setup levels 0..{args.level}: fine {nF} nodes / {cF} cells, {setup_s:.1f} s")
    for l in range(args.level + 1):
        log(f"workgroup sizes level {l}: {ctx.launch_config(l)}")

    # ---- full-depth GMG on the fine level (reference and baseline)
    sf = ctx.state(args.level)
    for k, s_ in enumerate(run_steps(ctx, sf, args.warmup, args.dt)):
        log(f"gmg warmup {k}: {s_}")
    ctx.profile_select(gmg_keys)
    ctx.profile_enable(True)
    stream.synchronize()
    t0 = time.perf_counter()
    g_stats = run_steps(ctx, sf, args.steps, args.dt)
    stream.synchronize()
    g_sec = time.perf_counter() - t0
    g_prof = ctx.profile_report()
    ctx.profile_enable(False)
    for k, s_ in enumerate(g_stats):
        log(f"gmg step {k}: {s_}")
    x_fine, _ = sf.get()

    # ---- DNN-MG: Newton-GMRES-MG on the coarse level + patch GRU on the fine level
    m = args.level - args.coarse_level
    net = P.Net(ctx, args.coarse_level, m, args.hidden, args.layers)
    nsteps = args.warmup + args.steps
    # fine reference at every step (untimed replay of the GMG run above)
    sfr = ctx.state(args.level)
    xF = [sfr.get()[0]]
    for _ in range(nsteps):
        ctx.step(sfr, args.dt)
        xF.append(sfr.get()[0])
    sfr.close()
    pre, post, coarse = (int(v) for v in args.dnnmg_sweeps.split(","))
    ctx.set_params(nu_pre=pre, nu_post=post, nu_coarse=coarse)   # coarse solves of the DNN-MG leg
    train_info = None
    if args.train_net:
        train_info = train_dnnmg(ctx, net, xF, args.coarse_level, args.dt, args.train_net_iters,
                                 args.dagger, args.seed, log)
    else:
        w = gru_weights(net.n_in, args.hidden, args.layers, net.n_out, seed=args.seed, scale=0.5)
        net.set_weights(w, mu=np.zeros(10), sigma=np.array([1, 1, 1, 10, 10, 10, 1, 1, 1, 100.0]),
                        out_scale=np.array([1e-3, 1e-3]))
    sc = ctx.state(args.coarse_level)
    net.reset(sc)
    for k, s_ in enumerate(run_steps(ctx, sc, args.warmup, args.dt, net)):
        log(f"dnnmg warmup {k}: {s_}")
    ctx.profile_select(dnn_keys)
    ctx.profile_enable(True)
    stream.synchronize()
    t0 = time.perf_counter()
    d_stats = run_steps(ctx, sc, args.steps, args.dt, net)
    stream.synchronize()
    d_sec = time.perf_counter() - t0
    d_prof = ctx.profile_report()
    ctx.profile_enable(False)
    for k, s_ in enumerate(d_stats):
        log(f"dnnmg step {k}: {s_}")
    sc.close()
    # velocity errors against the fine solution at every timed step (untimed
    # replays of the same deterministic runs)
    err_dnn, err_mgl = [], []
    n_obs = len(macro.curves)
    funcs = {}

    def fdict(x):
        j, d, lf = ctx.functionals(args.level, x, n_obs)
        return {"j_div": j, "drag": float(d[0]), "lift": float(lf[0])}
    for with_net in (True, False):
        st = ctx.state(args.coarse_level)
        if with_net:
            net.reset(st)
        for n in range(1, nsteps + 1):
            ctx.step(st, args.dt)
            xl, _ = st.get()
            corr = net.correct(st, args.dt, debug=True)["correction"] if with_net else None
            if n > args.warmup:
                e = velocity_error(ctx, xl, args.coarse_level, args.level, xF[n], corr)
                (err_dnn if with_net else err_mgl).append(e)
            if n == nsteps:   # functionals of the last step (Sec. 3.3)
                funcs["dnnmg" if with_net else "mg_coarse"] = fdict(
                    fine_state(ctx, xl, args.coarse_level, args.level, corr))
        st.close()
    funcs["reference_fine_gmg"] = fdict(xF[nsteps])
    err_dnn, err_mgl = float(np.mean(err_dnn)), float(np.mean(err_mgl))
    log(f"velocity error (mean over timed steps): DNN-MG {err_dnn:.3e}, MG(L) {err_mgl:.3e}")
    log(f"functionals at t = {nsteps * args.dt:.3f}: {funcs}")

    for name, prof in (("gmg", g_prof), ("dnnmg", d_prof)):
        for key in sorted(prof, key=lambda k: -prof[k][1])[:14]:
            cnt, ms = prof[key]
            log(f"{name} kernel {key}: {cnt} launches, {ms:.2f} ms total, {1e3 * ms / cnt:.1f} us avg")
    roof = roofline_from(g_prof, ctx, args.level, ("spmv", "residual_spmv", "vanka_apply", "vanka_update"),
                         log)
    # MFMA utilisation of the network's input GEMM (layer 0)
    mfma = None
    mkey = f"gru_gemm_in0@L{F}"
    if mkey in d_prof:
        cnt, ms = d_prof[mkey]
        flop = 2.0 * net.n_patches * 3 * args.hidden * ((net.n_in + 31) // 32 * 32)
        tf = flop / (ms / cnt / 1e3) / 1e12
        mfma = {"kernel": mkey, "achieved": round(tf, 2), "peak": 2500.0,
                "unit": "TFLOP/s", "frac": round(tf / 2500.0, 5), "avg_us": round(1e3 * ms / cnt, 2)}
    # ---- batched plain solves
    batch_info = run_batch(P, args, log) if args.batch_sims > 0 else None
    # ---- network-size sweep (Table 1 / Table 2 analogue)
    table1 = run_table1(P, args, log) if args.table1 else None
    # ---- BPTT training throughput at the training batch shape (synthetic rows)
    train = None
    if args.train_iters > 0:
        T, B = args.train_seq, args.train_batch
        gX = torch.randn(T, B, net.n_in, device="cuda", dtype=torch.float32)
        gD = 0.1 * torch.randn(T, B, net.n_out, device="cuda", dtype=torch.float32)
        torch.cuda.synchronize()
        net.train_step_dev(gX.data_ptr(), gD.data_ptr(), T, B, lr=1e-4, ckpt=8)   # warm-up / allocation
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.train_iters):
            net.train_step_dev(gX.data_ptr(), gD.data_ptr(), T, B, lr=1e-4, ckpt=8)
        stream.synchronize()
        tsec = (time.perf_counter() - t0) / args.train_iters
        H, I, O, Lr = args.hidden, net.n_in, net.n_out, args.layers
        fwd = 2.0 * (3 * H * ((I + 31) // 32 * 32) + 3 * H * H + (Lr - 1) * 6 * H * H + O * H)
        nseg = (T + 7) // 8                   # checkpoints every 8 steps
        # forward, recompute of all segments but the last, backward (2x forward)
        flop = T * B * fwd * (1 + (nseg - 1) / nseg + 2)
        train = {"seq": T, "batch": B, "hidden": H, "layers": Lr, "ms_per_iter": round(1e3 * tsec, 2),
                 "model_tflop_per_iter": round(flop / 1e12, 4),
                 "tflops": round(flop / tsec / 1e12, 2), "mfma_frac": round(flop / tsec / 2.5e15, 5)}
        log(f"train: {train}")
        del gX, gD

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.seed, args.cpu_level, args.level, args.dt)
    ms_step = 1e3 * d_sec / args.steps
    result = {
        "metric": METRIC,
        "value": round(args.steps / d_sec, 4),
        "unit": "time steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64+bf16",
        "data": "synthetic",
        "config": {"workload": (f"DNN-MG: Newton-GMRES-GMG on level {args.coarse_level} + GRU "
                                f"{args.hidden}x{args.layers} patch net correcting level {args.level}; "
                                f"channel+obstacle seed {args.seed}, Re 100, dt {args.dt}, mixed precision"),
                   "coarse_level": args.coarse_level, "fine_level": args.level,
                   "fine_dofs": 3 * nF, "coarse_dofs": 3 * nL, "patches": net.n_patches,
                   "gmg_steps_per_s": round(args.steps / g_sec, 4),
                   "gmg_ms_per_step": round(1e3 * g_sec / args.steps, 3),
                   "dnnmg_speedup_vs_gmg": round(g_sec / d_sec, 3),
                   "velocity_rel_l2_err_dnnmg": round(err_dnn, 6),
                   "velocity_rel_l2_err_mg_coarse": round(err_mgl, 6),
                   "net": "trained on the GPU (teacher forcing + DAgger)" if train_info else "random init",
                   "net_training": train_info,
                   "gmg_dof_updates_per_s": round(3 * nF * args.steps / g_sec, 1),
                   "gmg_newton_iters": sum(s_["newton_iters"] for s_ in g_stats),
                   "gmg_gmres_iters": sum(s_["gmres_iters"] for s_ in g_stats),
                   "gmg_jacobian_builds": sum(s_["jacobian_builds"] for s_ in g_stats),
                   "dnnmg_newton_iters": sum(s_["newton_iters"] for s_ in d_stats),
                   "dnnmg_gmres_iters": sum(s_["gmres_iters"] for s_ in d_stats),
                   "dnnmg_jacobian_builds": sum(s_["jacobian_builds"] for s_ in d_stats),
                   "dnnmg_fallbacks": sum(s_["fallback"] for s_ in d_stats),
                   "functionals_last_step": funcs,
                   "graphs": not args.no_graphs, "profile": args.profile,
                   "newton_predictor": args.newton_predictor,
                   "jacobian_reuse": args.jacobian_reuse, "smoother": args.smoother, "direct_solve_level": args.direct_level,
                   "v_cycle": {"gmg": f"V(2,2), {args.nu_coarse or 'same'} below the top",
                               "dnnmg": "V({},{}), V({c},{c}) below the top".format(
                                   *args.dnnmg_sweeps.split(",")[:2], c=args.dnnmg_sweeps.split(",")[2])}},
        "roofline": roof,
        "mfma": mfma,
        "train": train,
        "batch": batch_info,
        "table1": table1,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
