"""Benchmark: time steps/s of DNN-MG against full-depth GMG on one MI355X, at
a stated velocity error against the fine solution.

Workload (seeded synthetic stand-in for the paper's flow around an obstacle,
Sec. 3.1): channel with one circular obstacle (seed 0), Re = 100, dt = 0.005,
mixed precision (FP32 smoother, transfers and Krylov vectors; FP64 Newton
residual, update, coarse solve and Gram-Schmidt dots).

1. Developed flow: the plain method on level 5 from rest to t_dev (past the
   inflow ramp), prolongated to level 7 and relaxed by a few level-7 steps.
   Every leg below starts from that state x7.
2. Network: the patch GRU (hidden 128, 2 layers, BF16 MFMA) is trained on the
   GPU (untimed) on other geometries of the training generator (seeds 200..,
   Re ~ U[80, 120], each spun up the same way): teacher-forced sequences
   (Sec. 3.1 training data, eq. loss) plus rounds that add the states of free
   DNN-MG runs carried on from round to round, with targets from one fine
   step started from each such state; the round whose weights give the
   lowest velocity error on a validation geometry (the generator's next
   seed, not trained on) is kept.  The evaluated geometry is never seen in
   training.
3. Timed legs (the benchmark contract): full-depth GMG on level 7, and DNN-MG
   (Newton-GMRES-GMG on level 5 + the network correcting level 7,
   Algorithm 1), W untimed + K timed steps each from x7.  `value` is the
   DNN-MG rate.
4. Evaluation window (untimed for the contract, each step clocked): the
   level-7 GMG reference, MG(5) and DNN-MG run E steps from x7; velocity
   errors (mass-weighted L2 and nodal) of MG(5) and DNN-MG against level 7,
   Newton / GMRES counts, Jacobian rebuilds, switch-offs and the sustained
   rate of each leg over the window; and the mixed-precision reference
   against the GPU FP64 mode for a few steps.

`roofline` comes from per-kernel HIP-event timings the library records on its
stream over the timed GMG steps (the dominant kernel by total time, its
launches of both forms merged); `cpu_baseline` times the FP64 oracle on the
host: the FP64 parity workload (level 3, 10 steps) in full on one core and,
as independent runs, on all cores (optionally also level-5 steps).
Optional legs: batched plain solves (--batch-sims, or alone with
--batch-only), the network-size sweep of Table 1 (--table1, or alone with
--table1-only), the switch-off study (--switchoff-study) and held-out
geometries (--extra-eval-seeds).
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


# profiling keys that time the same kernel (merged for the roofline)
KERNEL_GROUPS = {"k_spmv": ("spmv", "residual_spmv"), "k_vanka_apply": ("vanka_apply",),
                 "k_vanka_update_ordered": ("vanka_update",)}


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




def roofline_from(prof, ctx, level, log=None):
    """Roofline of the kernel with the largest total time among the level's
    streaming kernels (launches under several profiling keys merged):
    achieved = algorithmic bytes / time over all its launches."""
    rows = []
    for kernel, keys in KERNEL_GROUPS.items():
        ms = cnt = 0
        nbytes = 0.0
        traffic = []
        for k in keys:
            key = f"{k}@L{level}"
            if key not in prof:
                continue
            c, t = prof[key]
            b = kernel_bytes(ctx, k, level)
            ms += t
            cnt += c
            nbytes += b * c
            traffic.append((measured_traffic(k, level), c))
        if cnt == 0:
            continue
        avg_s = ms / cnt / 1e3
        per_launch = nbytes / cnt
        if traffic and all(t is not None for t, _ in traffic):
            meas = int(sum(t * c for t, c in traffic) / sum(c for _, c in traffic))
        else:
            meas = None
        rows.append((ms, kernel, cnt, avg_s, per_launch, meas, keys))
        if log:
            log(f"roofline {kernel}@L{level} ({', '.join(keys)}): {cnt} launches, {ms:.1f} ms, "
                f"{per_launch / 1e6:.1f} MB/launch algorithmic, {avg_s * 1e6:.1f} us, "
                f"{per_launch / avg_s / 1e9:.0f} GB/s, measured traffic {meas}")
    if not rows:
        return None
    ms, kernel, cnt, avg_s, b, meas, keys = max(rows)
    ach = b / avg_s / 1e9
    return {"bound": "hbm", "kernel": f"{kernel}@L{level}", "profile_keys": list(keys),
            "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": meas, "avg_us": round(avg_s * 1e6, 2), "launches": cnt,
            "total_ms": round(ms, 2), "bytes_per_launch": int(b)}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_run(job):
    """Plain FP64 oracle run (Newton with direct sparse solves) on one core:
    (seed, level, dt, steps) -> (seconds, DoFs, Newton iterations)."""
    seed, level, dt, steps = job
    from threadpoolctl import threadpool_limits
    import numpy as np

    from oracle import fem, mesh, solver
    from synthetic import channel_obstacle
    macro = channel_obstacle(seed)
    L = mesh.hierarchy(macro, level)[level]
    prob = fem.Problem(nu=macro.nu, dt=dt)
    x = np.zeros(3 * L.n_nodes)
    newton = 0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for n in range(1, steps + 1):
            x, hist = solver.newton_step(L, prob, x, n * dt, tol=1e-10, return_history=True)
            newton += len(hist) - 1
        sec = time.perf_counter() - t0
    return sec, 3 * L.n_nodes, newton


def cpu_baseline(args, log):
    """The FP64 oracle on the host's cores.  The FP64 parity workload (seed 0,
    level 3, dt 0.01, 10 steps from rest) in full on one core; the same run for seeds 0..P-1 as P independent single-core processes
    (all cores); optionally level-5 steps of the same geometry (dt 0.005)."""
    import multiprocessing as mp
    nproc = os.cpu_count() or 1
    sec, dofs, newton = _oracle_run((0, 3, 0.01, 10))
    out = {"value": round(10 / sec, 4), "unit": "time steps/s", "cores": 1, "kind": "oracle",
           "sample": (f"the FP64 parity workload in full: FP64 oracle (numpy einsum assembly, SuperLU direct solves), seed 0, "
                      f"level 3 ({dofs} DoFs), dt 0.01, 10 steps from rest, {newton} Newton iterations, "
                      f"{sec:.2f} s on one core; not the headline's level-5/7 workload (one oracle DNN-MG "
                      f"step there takes minutes)"),
           "dof_updates_per_s": round(dofs * 10 / sec, 1), "nproc": nproc, "cpu_model": _cpu_model()}
    procs = max(1, min(args.cpu_procs, nproc))
    if procs > 1:
        jobs = [(s, 3, 0.01, 10) for s in range(procs)]
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(procs) as pool:
            res = pool.map(_oracle_run, jobs)
        wall = time.perf_counter() - t0
        out["all_cores"] = {"processes": procs, "threads_per_process": 1, "seeds": f"0..{procs - 1}",
                            "steps_per_s": round(10 * procs / wall, 4),
                            "dof_updates_per_s": round(sum(r[1] for r in res) * 10 / wall, 1),
                            "wall_s": round(wall, 2)}
    if args.cpu_c2_steps > 0:
        sec5, dofs5, newton5 = _oracle_run((0, 5, args.dt, args.cpu_c2_steps))
        out["level5"] = {"steps": args.cpu_c2_steps, "dofs": dofs5, "seconds": round(sec5, 2),
                         "steps_per_s": round(args.cpu_c2_steps / sec5, 5), "newton_iters": newton5,
                         "cores": 1}
    log(f"cpu baseline: {out}")
    return out


def run_steps(ctx, st, steps, dt, net=None):
    """`steps` time steps (plain, or DNN-MG: coarse step + correction)."""
    stats = []
    for _ in range(steps):
        stats.append(ctx.step(st, dt))
        if net is not None:
            net.correct(st, dt)
    return stats


def fine_state(ctx, xl, level, fine_level, corr=None):
    """P^m x^L on the fine level (host), with the network's velocity
    correction added."""
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
    the fine solution (host arrays; used by the small network-size sweep)."""
    import numpy as np
    v = fine_state(ctx, xl, level, fine_level, corr).reshape(-1, 3)[:, :2]
    ref = x_fine.reshape(-1, 3)[:, :2]
    return float(np.linalg.norm(v - ref) / np.linalg.norm(ref))


def make_context(P, macro, args, stream, precision=1):
    return P.Context(precision=precision, nu=macro.nu, stream=stream,
                     use_graphs=0 if args.no_graphs else 1, newton_predictor=args.newton_predictor,
                     jacobian_reuse=args.jacobian_reuse, smoother=args.smoother, nu_coarse=args.nu_coarse,
                     coarse_level=args.direct_level)


def spin_up(ctx, L, F, t_dev, relax, dt, log, tag):
    """Developed flow: the plain method on level L from rest to t_dev,
    prolongated to level F and relaxed by `relax` level-F steps; returns the
    host state on level F and its time."""
    sc = ctx.state(L)
    n = int(round(t_dev / dt))
    t0 = time.perf_counter()
    newton = 0
    for _ in range(n):
        newton += ctx.step(sc, dt)["newton_iters"]
    xl, t = sc.get()
    sc.close()
    sf = ctx.state(F)
    sf.set(fine_state(ctx, xl, L, F), t)
    for _ in range(relax):
        ctx.step(sf, dt)
    x, t = sf.get()
    sf.close()
    log(f"{tag}: level-{L} run from rest, {n} steps to t = {n * dt:.3f} ({newton} Newton iterations), "
        f"prolongated to level {F} and relaxed by {relax} steps, {time.perf_counter() - t0:.1f} s")
    return x, t


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
    and their per-column expansions.  Xr, Dr: lists of (T, B, .) arrays."""
    import numpy as np
    S2 = net.n_out // 2
    nch = (net.n_in - net.n_stats) // (S2 - 1)        # nodal channels (6 block, 5 cell)
    nft = net.n_stats - nch
    cols = [slice(c * S2, (c + 1) * S2) for c in range(nch)] + [slice(nch * S2 + k, nch * S2 + k + 1)
                                                                for k in range(nft)]

    def moments(arrs, sl):
        n = sum(a[..., sl].size for a in arrs)
        mean = sum(float(a[..., sl].sum(dtype=np.float64)) for a in arrs) / n
        var = sum(float(((a[..., sl].astype(np.float64) - mean) ** 2).sum()) for a in arrs) / n
        return mean, np.sqrt(var)

    st = [moments(Xr, sl) for sl in cols]
    mu = np.array([m for m, _ in st])
    sg = np.array([s for _, s in st])
    sg = np.where(sg > 1e-30, sg, 1.0)
    osc = np.array([moments(Dr, slice(0, S2))[1], moments(Dr, slice(S2, 2 * S2))[1]])
    osc = np.where(osc > 1e-30, osc, 1.0)
    mu_f = np.concatenate([np.repeat(mu[:nch], S2), mu[nch:]]).astype(np.float32)
    sg_f = np.concatenate([np.repeat(sg[:nch], S2), sg[nch:]]).astype(np.float32)
    os_f = np.concatenate([np.repeat(osc[0], S2), np.repeat(osc[1], S2)]).astype(np.float32)
    return (mu, sg, osc), (mu_f, sg_f, os_f)


def sequences(A, seq):
    """(T, B, n) -> (seq, (T // seq) B, n): consecutive windows of `seq` steps
    of every patch as separate sequences."""
    import numpy as np
    T = A.shape[0] // seq * seq
    A = A[:T].reshape(T // seq, seq, *A.shape[1:])
    return np.ascontiguousarray(A.transpose(1, 0, 2, 3).reshape(seq, -1, A.shape[-1]))


class Minibatches:
    """Device-resident training sequences in minibatch-major layout
    (nb, seq, B, n): each minibatch is contiguous, as the training entry point
    takes it (T x B rows, step-major).  Sequences are shuffled into
    minibatches with a seeded permutation; the remainder is dropped.  Only
    the shuffled copy is kept: added sequences are joined to it and the whole
    set is shuffled again."""

    def __init__(self, X, D, batch, seed):
        self.batch, self.seed = batch, seed
        self.build(X, D)

    def add(self, X, D):
        import torch
        seq = self.Xm.shape[1]

        def flat(A):
            return A.permute(1, 0, 2, 3).reshape(seq, -1, A.shape[3])
        X = torch.cat([flat(self.Xm), X], dim=1)
        del self.Xm
        D = torch.cat([flat(self.Dm), D], dim=1)
        del self.Dm
        self.build(X, D)

    def build(self, X, D):
        import torch
        seq, tot = X.shape[0], X.shape[1]
        B = min(self.batch, tot)
        self.nb = tot // B
        self.n_seq = self.nb * B
        g = torch.Generator(device="cpu").manual_seed(self.seed + tot)
        perm = torch.randperm(tot, generator=g)[:self.n_seq].to(X.device)

        def mb(A):
            return A.index_select(1, perm).reshape(seq, self.nb, B, A.shape[2]).permute(1, 0, 2, 3).contiguous()
        self.Xm = mb(X)
        del X
        self.Dm = mb(D)
        self.B = B

    def fit(self, net, iters, lr, ckpt=8):
        """Adam iterations over the minibatches in turn (lr drops to 0.3 lr for
        the last quarter); returns (last loss, seconds, iterations)."""
        import torch
        seq = self.Xm.shape[1]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = None
        for it in range(iters):
            k = it % self.nb
            loss = net.train_step_dev(self.Xm[k].data_ptr(), self.Dm[k].data_ptr(), seq, self.B,
                                      lr=lr if it < 0.75 * iters else 0.3 * lr, ckpt=min(ckpt, seq))
        torch.cuda.synchronize()
        return loss, time.perf_counter() - t0, iters


def train_on_geometries(P, args, log, stream):
    """Training workload (seeded geometries of the training generator, a
    reduced count): for each seed of the training generator, the developed
    flow on level F, a fine
    trajectory of train_steps steps, teacher-forced coarse steps (inputs and
    targets), then BPTT + Adam on the GPU; `dagger` rounds add the states of
    free DNN-MG runs on the same geometries, each step's target the
    correction that one fine step started from the run's own fine state gives
    (targets from the original fine trajectory would ask the network to undo
    the run's accumulated drift in one step).  The free run of a geometry
    starts at the start of its fine trajectory and each round carries it on
    from where the previous round stopped (coarse state, hidden state and
    corrected fine state kept), so the last round's states lie as far from
    the start as the evaluation window's.  With `val_steps`, a validation
    geometry of the same generator (the next seed, not trained on) is run
    with the weights of every round (teacher forcing, then each free-run
    round) against its own level-F trajectory, and the weights with the
    lowest mean velocity error there are returned.  Returns the trained
    weights, standardisation and a summary."""
    import numpy as np
    import torch

    from synthetic import gru_weights, training_channel
    L, F, dt, seq = args.coarse_level, args.level, args.dt, args.train_seq
    m = F - L
    geoms, Xr, Dr = [], [], []
    t_all = time.perf_counter()
    for k in range(args.train_geoms):
        seed = args.train_seed0 + k
        macro = training_channel(seed)
        ctx = make_context(P, macro, args, stream.cuda_stream)
        ctx.setup_mesh(macro, F)
        net = P.Net(ctx, L, m, args.hidden, args.layers)
        # staggered start times, so that the training states cover the evaluation window
        x0, t0 = spin_up(ctx, L, F, args.t_dev + args.train_stagger * k, args.relax, dt, log,
                         f"train seed {seed} (Re {0.1 / macro.nu:.1f})")
        sf = ctx.state(F)
        sf.set(x0, t0)
        xF = [x0]
        for _ in range(args.train_steps):
            ctx.step(sf, dt)
            xF.append(sf.get()[0])
        sf.close()
        X, D = teacher_data(ctx, net, xF, L, dt, t0=t0)
        Xr.append(X)
        Dr.append(D)
        geoms.append({"seed": seed, "re": round(0.1 / macro.nu, 2), "ctx": ctx, "net": net, "xF": xF, "t0": t0})
        log(f"train seed {seed}: {args.train_steps} fine steps + teacher-forced coarse steps, "
            f"{X.shape[1]} patches, {time.perf_counter() - t_all:.1f} s so far")
    net0 = geoms[0]["net"]
    (mu, sg, osc), (mu_f, sg_f, os_f) = standardisation(net0, Xr, Dr)
    val = None
    if args.val_steps > 0:
        vseed = args.train_seed0 + args.train_geoms
        vmacro = training_channel(vseed)
        vctx = make_context(P, vmacro, args, stream.cuda_stream)
        vctx.setup_mesh(vmacro, F)
        vnet = P.Net(vctx, L, m, args.hidden, args.layers)
        vx0, vt0 = spin_up(vctx, L, F, args.t_dev + args.train_stagger * args.train_geoms, args.relax, dt, log,
                           f"validation seed {vseed} (Re {0.1 / vmacro.nu:.1f})")
        vref = torch.empty((args.val_steps, 3 * vctx.level_info(F)[0]), dtype=torch.float64, device="cuda")
        sf = vctx.state(F)
        sf.set(vx0, vt0)
        for n in range(args.val_steps):
            vctx.step(sf, dt)
            sf.get_dev(vref[n].data_ptr())
        stream.synchronize()
        sf.close()
        val = {"seed": vseed, "re": round(0.1 / vmacro.nu, 2), "t_start": vt0, "ctx": vctx, "net": vnet,
               "x0": vx0, "ref": vref}

    def validate(w):
        """Mean mass-weighted velocity error of a free DNN-MG run with
        weights w on the validation geometry."""
        vctx, vnet = val["ctx"], val["net"]
        vnet.set_weights(w, mu=mu, sigma=sg, out_scale=osc)
        st = vctx.state(L)
        st.set(val["x0"][:3 * vctx.level_info(L)[0]], val["t_start"])
        vnet.reset(st)
        vnet.rhs_from_fine(st, val["x0"], dt)
        errs = []
        for n in range(args.val_steps):
            vctx.step(st, dt)
            vnet.correct(st, dt)
            errs.append(rel_errors(vctx.velocity_error(F, vnet.fine_velocity_ptr(), F,
                                                       val["ref"][n].data_ptr()))["l2"])
        st.close()
        return float(np.mean(errs))
    dev = torch.device("cuda")
    Xd = torch.cat([torch.from_numpy(sequences((X - mu_f) / sg_f, seq)).to(dev) for X in Xr], dim=1)
    Dd = torch.cat([torch.from_numpy(sequences(D / os_f, seq)).to(dev) for D in Dr], dim=1)
    del Xr, Dr
    data = Minibatches(Xd, Dd, args.train_batch, args.seed)
    del Xd, Dd
    w0 = gru_weights(net0.n_in, args.hidden, args.layers, net0.n_out, seed=args.seed, scale=0.5)
    net0.set_weights(w0, mu=mu, sigma=sg, out_scale=osc)
    loss, sec, its = data.fit(net0, args.train_net_iters, 2e-3)
    fit_sec, fit_its = sec, its
    log(f"net training (teacher forcing): loss {loss:.2f}, {data.n_seq} sequences of {seq} steps, "
        f"{data.nb} minibatches of {data.B}, {1e3 * sec / its:.2f} ms per iteration")
    val_err, best = [], None
    if val:
        w = net0.get_weights()
        val_err.append(validate(w))
        best = (val_err[-1], 0, w)
        log(f"validation (teacher forcing): mean velocity error {val_err[-1]:.3e}")
    runs = {}
    for rnd in range(args.dagger):
        # free DNN-MG runs with the current network; the target of each step is
        # the correction that one fine step, started from the run's own fine
        # state (the corrected velocity of the previous step), gives
        w = net0.get_weights()
        Xc_all, Dc_all = [], []
        for i, g in enumerate(geoms):
            ctx, net = g["ctx"], g["net"]
            if net is not net0:
                net.set_weights(w, mu=mu, sigma=sg, out_scale=osc)
            if i not in runs:
                # the free run starts where the geometry's fine trajectory starts
                x0, t0 = g["xF"][0], g["t0"]
                nL = ctx.level_info(L)[0]
                st = ctx.state(L)
                st.set(x0[:3 * nL], t0)
                net.reset(st)
                net.rhs_from_fine(st, x0, dt)
                runs[i] = [st, ctx.state(F), x0]
            st, sf, vc = runs[i]
            Xc, Dc = [], []
            for n in range(args.dagger_steps):
                t = st.get()[1]
                sf.set(vc, t)
                ctx.step(sf, dt)
                xstar = sf.get()[0]
                ctx.step(st, dt)
                out = net.correct(st, dt, debug=True)
                Xc.append(out["inputs"])
                Dc.append(net.targets(st, xstar))
                xt = fine_state(ctx, st.get()[0], L, F).reshape(-1, 3).copy()
                xt[:, :2] += out["correction"]
                vc = xt.reshape(-1)
            runs[i][2] = vc
            Xc_all.append(torch.from_numpy(sequences(np.stack(Xc), seq)).to(dev))
            Dc_all.append(torch.from_numpy(sequences(np.stack(Dc), seq)).to(dev))
            log(f"free-run round {rnd + 1}, seed {g['seed']}: {args.dagger_steps} steps, "
                f"{time.perf_counter() - t_all:.1f} s so far")
        data.add(torch.cat(Xc_all, dim=1), torch.cat(Dc_all, dim=1))
        loss, sec, its = data.fit(net0, args.dagger_iters, 1e-3)
        fit_sec += sec
        fit_its += its
        log(f"net training (round {rnd + 1}, free DNN-MG states added): loss {loss:.2f}, "
            f"{data.n_seq} sequences")
        if val:
            w = net0.get_weights()
            val_err.append(validate(w))
            if val_err[-1] < best[0]:
                best = (val_err[-1], rnd + 1, w)
            log(f"validation (round {rnd + 1}): mean velocity error {val_err[-1]:.3e}")
    for st, sf, _ in runs.values():
        sf.close()
        st.close()
    w = best[2] if val else net0.get_weights()
    info = {"geometries": [{"seed": g["seed"], "re": g["re"]} for g in geoms],
            "t_start": [round(g["t0"], 4) for g in geoms], "fine_steps_per_geometry": args.train_steps,
            "sequences": int(data.n_seq), "seq": seq, "batch": data.B, "rounds": 1 + args.dagger,
            "free_run_steps_per_round": args.dagger_steps,
            "free_run_horizon_steps": args.dagger * args.dagger_steps,
            "adam_iters": fit_its, "final_loss": round(float(loss), 4),
            "bptt_ms_per_iter": round(1e3 * fit_sec / fit_its, 3),
            "wall_s": round(time.perf_counter() - t_all, 1)}
    if val:
        info["validation"] = {"seed": val["seed"], "re": val["re"], "t_start": round(val["t_start"], 4),
                              "steps": args.val_steps, "mean_l2_per_round": [float(f"{e:.4e}") for e in val_err],
                              "kept_round": best[1]}
        val["net"].close()
        val["ctx"].close()
        del val["ref"]
    for g in geoms:
        g["net"].close()
        g["ctx"].close()
    del data
    torch.cuda.empty_cache()
    return w, (mu, sg, osc), info


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
        (mu, sg, osc), (mu_f, sg_f, os_f) = standardisation(net, [Xr], [Dr])
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




def eval_geometry(P, args, macro, net_state, log, stream, tag):
    """Error window on another geometry (held-out evaluation): developed flow,
    the level-F reference over eval_steps steps, then MG(L), DNN-MG with the
    trained network and DNN-MG with d = 0 over the same window; mean / last
    mass-weighted and nodal errors of each against the reference."""
    import numpy as np
    import torch
    L, F, dt, E = args.coarse_level, args.level, args.dt, args.eval_steps
    pre, post, coarse = (int(v) for v in args.dnnmg_sweeps.split(","))
    w_net, mu, sg, osc = net_state
    ctx = make_context(P, macro, args, stream.cuda_stream)
    ctx.setup_mesh(macro, F)
    nF, nL = ctx.level_info(F)[0], ctx.level_info(L)[0]
    x7, t7 = spin_up(ctx, L, F, args.t_dev, args.relax, dt, log, tag)
    ref = torch.empty((E, 3 * nF), dtype=torch.float64, device="cuda")
    sf = ctx.state(F)
    sf.set(x7, t7)
    for n in range(E):
        ctx.step(sf, dt)
        sf.get_dev(ref[n].data_ptr())
    stream.synchronize()
    sf.close()
    ctx.set_params(nu_pre=pre, nu_post=post, nu_coarse=coarse)
    out = {"re": round(0.1 / macro.nu, 2), "obstacles": int(len(macro.curves)), "t_start": round(t7, 4)}
    sc = ctx.state(L)
    sc.set(x7[:3 * nL], t7)
    errs, newton = [], []
    for n in range(E):
        newton.append(ctx.step(sc, dt)["newton_iters"])
        errs.append(rel_errors(ctx.velocity_error(L, sc.device_ptr(), F, ref[n].data_ptr())))
    sc.close()
    out["mg_coarse"] = err_summary(errs)
    n_off = max(1, int(round(2 * np.median(newton[:10]))))
    ctx.set_params(nu_pre=pre, nu_post=post, nu_coarse=coarse, switch_off_newton=n_off)
    for name, weights in (("dnnmg", w_net), ("dnnmg_zero_net", None)):
        net = P.Net(ctx, L, F - L, args.hidden, args.layers)
        if weights is None:
            net.set_weights(np.zeros(net.n_params, dtype=np.float32), mu=np.zeros(10), sigma=np.ones(10),
                            out_scale=np.ones(2))
        else:
            net.set_weights(weights, mu=mu, sigma=sg, out_scale=osc)
        sc = ctx.state(L)
        sc.set(x7[:3 * nL], t7)
        net.reset(sc)
        net.rhs_from_fine(sc, x7, dt)
        errs, fallbacks = [], 0
        for n in range(E):
            fallbacks += ctx.step(sc, dt)["fallback"]
            net.correct(sc, dt)
            errs.append(rel_errors(ctx.velocity_error(F, net.fine_velocity_ptr(), F, ref[n].data_ptr())))
        sc.close()
        net.close()
        out[name] = dict(err_summary(errs), fallbacks=fallbacks)
    del ref
    ctx.close()
    torch.cuda.empty_cache()
    log(f"{tag}: {out}")
    return out


def clocked(stream, fn):
    """Runs fn() between two stream synchronisations; (result, seconds)."""
    stream.synchronize()
    t0 = time.perf_counter()
    r = fn()
    stream.synchronize()
    return r, time.perf_counter() - t0


def err_summary(errs):
    import numpy as np
    out = {}
    for k in ("l2", "nodal"):
        v = np.array([e[k] for e in errs])
        out[f"{k}_mean"] = round(float(v.mean()), 7)
        out[f"{k}_max"] = round(float(v.max()), 7)
        out[f"{k}_last"] = round(float(v[-1]), 7)
    return out


def rel_errors(e):
    import math
    return {"l2": math.sqrt(e["l2_err2"] / e["l2_ref2"]), "nodal": math.sqrt(e["nodal_err2"] / e["nodal_ref2"])}


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
    ap.add_argument("--seed", type=int, default=0, help="evaluated geometry (channel_obstacle seed)")
    ap.add_argument("--t-dev", type=float, default=3.0,
                    help="developed flow: the level-L run from rest reaches this time before the legs start")
    ap.add_argument("--relax", type=int, default=10, help="level-F steps after prolongating the level-L state")
    ap.add_argument("--eval-steps", type=int, default=200,
                    help="evaluation window: steps of the reference, MG(L) and DNN-MG runs from the start state")
    ap.add_argument("--fp64-steps", type=int, default=5,
                    help="steps of the GPU FP64 mode compared with the mixed-precision reference")
    ap.add_argument("--train-net", type=int, default=1, choices=(0, 1),
                    help="train the patch network on held-out geometries (untimed); 0: random weights")
    ap.add_argument("--train-geoms", type=int, default=4, help="training geometries (seeds train-seed0..)")
    ap.add_argument("--train-seed0", type=int, default=200)
    ap.add_argument("--train-stagger", type=float, default=0.25,
                    help="training geometry k starts its fine trajectory at t_dev + k * stagger")
    ap.add_argument("--train-steps", type=int, default=64, help="fine steps per training geometry")
    ap.add_argument("--train-seq", type=int, default=32)
    ap.add_argument("--train-batch", type=int, default=8192)
    ap.add_argument("--train-net-iters", type=int, default=1500, help="Adam iterations on the teacher-forced data")
    ap.add_argument("--dagger", type=int, default=3,
                    help="training rounds on free DNN-MG runs of the training geometries (targets from one "
                         "fine step started from the run's own state; each round carries the runs on)")
    ap.add_argument("--dagger-steps", type=int, default=64, help="free-run steps per geometry and round")
    ap.add_argument("--dagger-iters", type=int, default=1000, help="Adam iterations after each free-run round")
    ap.add_argument("--val-steps", type=int, default=200,
                    help="steps of the validation run (training generator seed train-seed0 + train-geoms, not "
                         "trained on) that picks the round whose weights are kept; 0: the last round's")
    ap.add_argument("--extra-eval-seeds", default="",
                    help="comma-separated channel seeds (e.g. 300,301,302,303) evaluated like the main "
                         "geometry (error window only) with the same trained network")
    ap.add_argument("--zero-net-control", type=int, default=1, choices=(0, 1),
                    help="also run the DNN-MG window with a zero network (d = 0): the coupling's own error")
    ap.add_argument("--switchoff-study", type=int, default=0, choices=(0, 1),
                    help="DNN-MG over the window for each switch-off threshold, trained and hostile network")
    ap.add_argument("--switchoff-thresholds", default="0,3,5,7,10")
    ap.add_argument("--hostile-scale", type=float, default=20.0,
                    help="hostile network: the trained weights with every correction scaled by this factor")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="independent single-core oracle runs for the all-cores figure (capped at nproc)")
    ap.add_argument("--cpu-c2-steps", type=int, default=0,
                    help="also time this many oracle steps on level 5 of the evaluated geometry")
    ap.add_argument("--profile", choices=("roofline", "all"), default="roofline",
                    help="roofline: HIP events only around the fine-level GMG kernels and "
                         "the network kernels; all: every kernel of every level, launched "
                         "directly (no graphs; events add launch overhead to the timings)")
    ap.add_argument("--newton-predictor", type=int, default=1, choices=(0, 1),
                    help="1: Newton starts from the linear extrapolation of the last two states")
    ap.add_argument("--jacobian-reuse", type=int, default=1, choices=(0, 1),
                    help="keep Newton's Jacobians across iterations and steps while the "
                         "residual contracts by 0.1 or better (0: rebuild every step)")
    ap.add_argument("--nu-coarse", type=int, default=0,
                    help="full-depth GMG leg: sweeps before and after on the V-cycle levels below the "
                         "one GMRES works on (0: the same V(2,2) on every level)")
    ap.add_argument("--dnnmg-sweeps", default="2,2,0",
                    help="pre,post,coarse sweeps of the V-cycles of the level-L solves (MG(L) and "
                         "DNN-MG legs; coarse 0: pre/post on every level, as the GMG leg's V(2,2))")
    ap.add_argument("--direct-level", type=int, default=1, choices=(0, 1, 2),
                    help="level of the direct (FP64 dense inverse) solve at the bottom of every V-cycle")
    ap.add_argument("--smoother", type=int, default=0, choices=(0, 1),
                    help="0: additive cell-Vanka, 1: coloured multiplicative cell-Vanka")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel directly instead of replaying captured graphs")
    ap.add_argument("--batch-sims", type=int, default=0,
                    help="batched plain solves: simulations (0 skips the leg)")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-only", action="store_true", help="run only the batched-solve leg")
    ap.add_argument("--table1-only", action="store_true", help="run only the network-size sweep")
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--table1", type=int, default=0, choices=(0, 1),
                    help="network-size sweep (Table 1 shapes on cell patches, untimed leg)")
    ap.add_argument("--t1-level", type=int, default=3)
    ap.add_argument("--t1-dt", type=float, default=0.01)
    ap.add_argument("--t1-train-from", type=float, default=4.0)
    ap.add_argument("--t1-start", type=float, default=7.0)
    ap.add_argument("--t1-end", type=float, default=10.0)
    ap.add_argument("--t1-iters", type=int, default=3000)
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

    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.calib_copy_mb > 0:
        src = torch.ones(args.calib_copy_mb * (1 << 18), device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    L, F, dt, W, K, E = args.coarse_level, args.level, args.dt, args.warmup, args.steps, args.eval_steps
    m = F - L
    pre, post, coarse = (int(v) for v in args.dnnmg_sweeps.split(","))
    if args.profile == "all":
        gmg_keys = dnn_keys = None
    else:
        gmg_keys = [f"{k}@L{F}" for k in ("spmv", "residual_spmv", "vanka_apply", "vanka_update",
                                          "assemble", "vanka_factor", "residual", "gs_dots")]
        dnn_keys = [f"{k}{l}@L{F}" for l in range(args.layers) for k in ("gru_gemm_in", "gru_step")]
        dnn_keys += [f"{k}@L{F}" for k in ("gru_head", "dnnmg_rhs", "dnnmg_prolong", "patch_gather",
                                           "patch_scatter")]

    if args.batch_only:     # only the batched-solve leg (profiling runs)
        print(json.dumps({"batch": run_batch(P, args, log)}), flush=True)
        return
    if args.table1_only:    # only the network-size sweep
        print(json.dumps({"table1": run_table1(P, args, log)}), flush=True)
        return

    # ---- network training on held-out geometries (untimed)
    train_info = None
    if args.train_net:
        w_net, (mu, sg, osc), train_info = train_on_geometries(P, args, log, stream)

    # ---- the evaluated geometry: developed flow on level F
    macro = channel_obstacle(args.seed)
    ctx = make_context(P, macro, args, stream.cuda_stream)
    t0 = time.perf_counter()
    ctx.setup_mesh(macro, F)
    setup_s = time.perf_counter() - t0
    nF, cF, _ = ctx.level_info(F)
    nL = ctx.level_info(L)[0]
    log(f"setup levels 0..{F}: fine {nF} nodes / {cF} cells, {setup_s:.1f} s")
    for lv in range(F + 1):
        log(f"workgroup sizes level {lv}: {ctx.launch_config(lv)}")
    x7, t7 = spin_up(ctx, L, F, args.t_dev, args.relax, dt, log, f"seed {args.seed}")
    net = P.Net(ctx, L, m, args.hidden, args.layers)
    if args.train_net:
        net.set_weights(w_net, mu=mu, sigma=sg, out_scale=osc)
    else:
        w = gru_weights(net.n_in, args.hidden, args.layers, net.n_out, seed=args.seed, scale=0.5)
        net.set_weights(w, mu=np.zeros(10), sigma=np.array([1, 1, 1, 10, 10, 10, 1, 1, 1, 100.0]),
                        out_scale=np.array([1e-3, 1e-3]))

    def start_coarse(with_net):
        st = ctx.state(L)
        st.set(x7[:3 * nL], t7)
        if with_net:
            net.reset(st)
            net.rhs_from_fine(st, x7, dt)     # the first correction starts from the fine state
        return st

    # ---- A. timed full-depth GMG on level F
    sf = ctx.state(F)
    sf.set(x7, t7)
    for k, s_ in enumerate(run_steps(ctx, sf, W, dt)):
        log(f"gmg warmup {k}: {s_}")
    ctx.profile_select(gmg_keys)
    ctx.profile_enable(True)
    g_stats, g_sec = clocked(stream, lambda: run_steps(ctx, sf, K, dt))
    g_prof = ctx.profile_report()
    ctx.profile_enable(False)
    sf.close()
    for k, s_ in enumerate(g_stats):
        log(f"gmg step {k}: {s_}")

    # ---- B. reference trajectory over the evaluation window (level F, on the device)
    ref = torch.empty((E, 3 * nF), dtype=torch.float64, device="cuda")
    sf = ctx.state(F)
    sf.set(x7, t7)
    ref_stats, ref_sec = [], 0.0
    for n in range(E):
        s_, sec = clocked(stream, lambda: ctx.step(sf, dt))
        ref_stats.append(s_)
        ref_sec += sec
        sf.get_dev(ref[n].data_ptr())
        if (n + 1) % 250 == 0 and n + 1 < E:
            log(f"reference: {n + 1} of {E} steps")
    stream.synchronize()
    sf.close()
    log(f"reference: {E} level-{F} steps, {E / ref_sec:.2f} steps/s sustained, "
        f"{sum(s['jacobian_builds'] for s in ref_stats)} hierarchy builds")

    # ---- C. GPU FP64 mode against the mixed-precision reference
    fp64 = None
    if args.fp64_steps > 0:
        c64 = make_context(P, macro, args, stream.cuda_stream, precision=0)
        c64.setup_mesh(macro, F)
        s64 = c64.state(F)
        s64.set(x7, t7)
        tmp = torch.empty(3 * nF, dtype=torch.float64, device="cuda")
        worst = {"u": 0.0, "v": 0.0, "p": 0.0}
        for n in range(min(args.fp64_steps, E)):
            c64.step(s64, dt)
            s64.get_dev(tmp.data_ptr())
            stream.synchronize()
            a, b = tmp.view(-1, 3), ref[n].view(-1, 3)
            for f, name in enumerate("uvp"):
                e = float(torch.linalg.norm(a[:, f] - b[:, f]) / torch.linalg.norm(b[:, f]))
                worst[name] = max(worst[name], e)
        fp64 = {"steps": min(args.fp64_steps, E), "max_rel_l2": {k: float(f"{v:.3e}") for k, v in worst.items()}}
        log(f"mixed precision vs GPU FP64 mode on level {F}: {fp64}")
        s64.close()
        c64.close()
        del tmp

    # ---- D. MG(L) over the window: errors against the reference
    ctx.set_params(nu_pre=pre, nu_post=post, nu_coarse=coarse)
    sc = start_coarse(False)
    mgl_stats, mgl_sec, mgl_err = [], 0.0, []
    for n in range(E):
        s_, sec = clocked(stream, lambda: ctx.step(sc, dt))
        mgl_stats.append(s_)
        mgl_sec += sec
        mgl_err.append(rel_errors(ctx.velocity_error(L, sc.device_ptr(), F, ref[n].data_ptr())))
        if (n + 1) % 500 == 0 and n + 1 < E:
            log(f"MG({L}): {n + 1} of {E} steps")
    sc.close()
    n_off = max(1, int(round(2 * np.median([s_["newton_iters"] for s_ in mgl_stats[:10]]))))
    ctx.set_params(nu_pre=pre, nu_post=post, nu_coarse=coarse, switch_off_newton=n_off)

    # ---- E. timed DNN-MG
    sc = start_coarse(True)
    for k, s_ in enumerate(run_steps(ctx, sc, W, dt, net)):
        log(f"dnnmg warmup {k}: {s_}")
    ctx.profile_select(dnn_keys)
    ctx.profile_enable(True)
    d_stats, d_sec = clocked(stream, lambda: run_steps(ctx, sc, K, dt, net))
    d_prof = ctx.profile_report()
    ctx.profile_enable(False)
    sc.close()
    for k, s_ in enumerate(d_stats):
        log(f"dnnmg step {k}: {s_}")

    def leg(stats, sec):
        return {"steps_per_s": round(len(stats) / sec, 3),
                "newton_iters": sum(s_["newton_iters"] for s_ in stats),
                "gmres_iters": sum(s_["gmres_iters"] for s_ in stats),
                "jacobian_builds": sum(s_["jacobian_builds"] for s_ in stats),
                "fallbacks": sum(s_["fallback"] for s_ in stats)}

    # ---- F. DNN-MG over the window (and, as a control, with d = 0)
    def dnnmg_window(the_net):
        sc = start_coarse(False)
        the_net.reset(sc)
        the_net.rhs_from_fine(sc, x7, dt)
        stats, total, errs = [], 0.0, []
        for n in range(E):
            def one():
                s_ = ctx.step(sc, dt)
                the_net.correct(sc, dt)
                return s_
            s_, sec = clocked(stream, one)
            stats.append(s_)
            total += sec
            errs.append(rel_errors(ctx.velocity_error(F, the_net.fine_velocity_ptr(), F, ref[n].data_ptr())))
            if (n + 1) % 500 == 0 and n + 1 < E:
                log(f"DNN-MG window: {n + 1} of {E} steps")
        sc.close()
        return stats, total, errs

    dnn_stats, dnn_sec, dnn_err = dnnmg_window(net)
    zero_err = None
    if args.zero_net_control:
        znet = P.Net(ctx, L, m, args.hidden, args.layers)
        znet.set_weights(np.zeros(znet.n_params, dtype=np.float32), mu=np.zeros(10), sigma=np.ones(10),
                         out_scale=np.ones(2))
        zero_err = dnnmg_window(znet)[2]
        znet.close()
    # ---- switch-off study (Sec. 3.3): DNN-MG over the window for a range of
    # Newton-count thresholds, with the trained network and a hostile one
    # (the same weights with every correction scaled by --hostile-scale)
    switchoff = None
    if args.switchoff_study:
        switchoff = {"thresholds": [int(v) for v in args.switchoff_thresholds.split(",")],
                     "hostile_scale": args.hostile_scale, "runs": []}
        hnet = P.Net(ctx, L, m, args.hidden, args.layers)
        w_cur = net.get_weights()
        hnet.set_weights(w_cur, mu=mu if args.train_net else np.zeros(10),
                         sigma=sg if args.train_net else np.array([1, 1, 1, 10, 10, 10, 1, 1, 1, 100.0]),
                         out_scale=(osc if args.train_net else np.array([1e-3, 1e-3])) * args.hostile_scale)
        for kind, the_net in (("trained", net), ("hostile", hnet)):
            for thr in switchoff["thresholds"]:
                ctx.set_params(nu_pre=pre, nu_post=post, nu_coarse=coarse, switch_off_newton=thr)
                st_, sec_, er_ = dnnmg_window(the_net)
                row = dict(net=kind, threshold=thr, **leg(st_, sec_), **{k: v for k, v in err_summary(er_).items()
                                                                      if k in ("l2_mean", "l2_last")})
                log(f"switch-off study: {row}")
                switchoff["runs"].append(row)
        hnet.close()
        ctx.set_params(nu_pre=pre, nu_post=post, nu_coarse=coarse, switch_off_newton=n_off)
    del ref
    err_d, err_l = err_summary(dnn_err), err_summary(mgl_err)
    err_z = err_summary(zero_err) if zero_err else None
    trace = {name: [round(e[n]["l2"], 7) for n in range(0, E, max(1, E // 10))] + [round(e[-1]["l2"], 7)]
             for name, e in (("dnnmg", dnn_err), ("mg_coarse", mgl_err), ("dnnmg_zero_net", zero_err)) if e}
    log(f"velocity error over {E} steps: DNN-MG {err_d}, MG({L}) {err_l}, DNN-MG with d = 0 {err_z}")
    log(f"l2 error trace (every {max(1, E // 10)} steps): {trace}")

    for name, prof in (("gmg", g_prof), ("dnnmg", d_prof)):
        for key in sorted(prof, key=lambda k: -prof[k][1])[:14]:
            cnt, ms = prof[key]
            log(f"{name} kernel {key}: {cnt} launches, {ms:.2f} ms total, {1e3 * ms / cnt:.1f} us avg")
    roof = roofline_from(g_prof, ctx, F, log)
    # MFMA utilisation of the network's input GEMM (layer 0)
    mfma = None
    mkey = f"gru_gemm_in0@L{F}"
    if mkey in d_prof:
        cnt, ms = d_prof[mkey]
        flop = 2.0 * net.n_patches * 3 * args.hidden * ((net.n_in + 31) // 32 * 32)
        tf = flop / (ms / cnt / 1e3) / 1e12
        mfma = {"kernel": mkey, "achieved": round(tf, 2), "peak": 2500.0,
                "unit": "TFLOP/s", "frac": round(tf / 2500.0, 5), "avg_us": round(1e3 * ms / cnt, 2)}
    train = None
    if train_info:
        H, I, O, Lr, T = args.hidden, net.n_in, net.n_out, args.layers, args.train_seq
        fwd = 2.0 * (3 * H * ((I + 31) // 32 * 32) + 3 * H * H + (Lr - 1) * 6 * H * H + O * H)
        nseg = (T + 7) // 8                   # checkpoints every 8 steps
        # forward, recompute of all segments but the last, backward (2x forward)
        flop = T * train_info["batch"] * fwd * (1 + (nseg - 1) / nseg + 2)
        tsec = train_info["bptt_ms_per_iter"] / 1e3
        train = {"seq": T, "batch": train_info["batch"], "hidden": H, "layers": Lr,
                 "ms_per_iter": train_info["bptt_ms_per_iter"], "data": "solver trajectories (training leg)",
                 "model_tflop_per_iter": round(flop / 1e12, 4), "tflops": round(flop / tsec / 1e12, 2),
                 "mfma_frac": round(flop / tsec / 2.5e15, 5)}
    net.close()
    ctx.close()
    torch.cuda.empty_cache()
    held_out = None
    if args.extra_eval_seeds and args.train_net:
        from synthetic import channel_obstacle as geom
        held_out = {s_: eval_geometry(P, args, geom(int(s_)), (w_net, mu, sg, osc), log, stream,
                                      f"held-out seed {s_}")
                    for s_ in args.extra_eval_seeds.split(",")}
    batch_info = run_batch(P, args, log) if args.batch_sims > 0 else None
    table1 = run_table1(P, args, log) if args.table1 else None
    cpu = None if args.no_cpu_baseline else cpu_baseline(args, log)
    result = {
        "metric": METRIC,
        "value": round(K / d_sec, 4),
        "unit": "time steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(1e3 * d_sec / K, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64+bf16",
        "data": "synthetic",
        "config": {"workload": (f"DNN-MG: Newton-GMRES-GMG on level {L} + GRU {args.hidden}x{args.layers} "
                                f"patch net correcting level {F}; channel+obstacle seed {args.seed}, Re 100, "
                                f"dt {dt}, developed flow from t = {t7:.3f}, mixed precision"),
                   "coarse_level": L, "fine_level": F, "fine_dofs": 3 * nF, "coarse_dofs": 3 * nL,
                   "patches": net.n_patches, "t_start": round(t7, 4),
                   "gmg_steps_per_s": round(K / g_sec, 4), "gmg_ms_per_step": round(1e3 * g_sec / K, 3),
                   "dnnmg_speedup_vs_gmg": round(g_sec / d_sec, 3),
                   "gmg_dof_updates_per_s": round(3 * nF * K / g_sec, 1),
                   "timed": {"gmg": leg(g_stats, g_sec), "dnnmg": leg(d_stats, d_sec)},
                   "eval_steps": E,
                   "velocity_rel_err": {"dnnmg": err_d, "mg_coarse": err_l, "dnnmg_zero_net": err_z,
                                        "l2_trace": trace,
                                        "norms": "l2: mass-weighted (2x2 Gauss) on level F; nodal: over "
                                                 "the level-F nodes; relative to the level-F reference"},
                   "velocity_rel_l2_err_dnnmg": err_d["l2_mean"],
                   "velocity_rel_l2_err_mg_coarse": err_l["l2_mean"],
                   "sustained": {"gmg": leg(ref_stats, ref_sec), "mg_coarse": leg(mgl_stats, mgl_sec),
                                 "dnnmg": leg(dnn_stats, dnn_sec)},
                   "switch_off_newton": n_off,
                   "held_out_geometries": held_out,
                   "switch_off_study": switchoff,
                   "mixed_vs_fp64": fp64,
                   "net": ("trained on the GPU on held-out geometries (teacher forcing + free-run rounds); "
                           "the evaluated geometry is not in the training set") if train_info else "random init",
                   "net_training": train_info,
                   "graphs": not args.no_graphs, "profile": args.profile,
                   "newton_predictor": args.newton_predictor, "jacobian_reuse": args.jacobian_reuse,
                   "smoother": args.smoother, "direct_solve_level": args.direct_level,
                   "v_cycle": {"gmg": f"V(2,2), {args.nu_coarse or 'same'} below the top",
                               "mg_coarse_and_dnnmg": f"V({pre},{post}), "
                                                      f"{f'V({coarse},{coarse})' if coarse else 'same'} below the top"}},
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
