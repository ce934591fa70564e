"""Scheduling-only features (GPU): graph replay of V-cycles and of the
level-0 Gauss-Jordan sweep, and the workgroup-size autotuner.

The library captures the launch sequence of a V-cycle (and of the coarse
inverse) once and replays it; the replay runs the same kernels in the same
order, so every result must be bitwise equal to direct launches.  Each check
replays a graph several times with direct (eager) work and synchronisations
in between, compares every replay, and covers the rebuild after the Vanka
damping changes (the damping is baked into the captured launches).
"""
import numpy as np
import pytest

from oracle import mesh
from synthetic import channel_obstacle, random_state

pytestmark = pytest.mark.gpu

DT = 0.01
LEVEL = 3


def _pair(precision, stream=None):
    import paper_2106_07687_amd as P
    macro = channel_obstacle(0)
    out = []
    for g in (1, 0):
        kw = dict(nu=macro.nu, use_graphs=g)
        if stream is not None and g == 1:
            kw["stream"] = stream
        ctx = P.Context(precision=precision, **kw)
        ctx.setup_mesh(macro, LEVEL)
        out.append(ctx)
    lev = mesh.hierarchy(macro, LEVEL)
    return out[0], out[1], lev


def _rhs(lev, l, seed):
    b = random_state(lev[l].n_nodes, seed)
    b.reshape(-1, 3)[lev[l].dirichlet_nodes(), :2] = 0.0
    return b


@pytest.mark.parametrize("precision", [1, 0])
def test_vcycle_replays_are_bitwise_equal(precision):
    cg, ce, lev = _pair(precision)
    x = random_state(lev[LEVEL].n_nodes, 3) * 0.3
    states = []
    for ctx in (cg, ce):
        st = ctx.state(LEVEL)
        st.set(x, 0.0)
        ctx.linearize(st, LEVEL, DT)
        states.append(st)
    for rep in range(3):
        for l in (LEVEL, 2, 1):
            b = _rhs(lev, l, 20 + rep)
            vg, ve = cg.vcycle(l, b), ce.vcycle(l, b)
            print(f"[graphs] precision {precision} replay {rep} level {l}", flush=True)
            assert np.array_equal(vg, ve), (rep, l, np.abs(vg - ve).max())
            # eager work between replays
            x0 = _rhs(lev, LEVEL, 40 + rep) * 0.1
            assert np.array_equal(cg.vanka_sweep(LEVEL, x0, _rhs(lev, LEVEL, 50)),
                                  ce.vanka_sweep(LEVEL, x0, _rhs(lev, LEVEL, 50)))
    # a parameter change must rebuild the captured sequences
    for ctx in (cg, ce):
        ctx.set_params(vanka_omega=0.5)
    b = _rhs(lev, LEVEL, 60)
    vg, ve = cg.vcycle(LEVEL, b), ce.vcycle(LEVEL, b)
    assert np.array_equal(vg, ve)
    for ctx in (cg, ce):
        ctx.set_params(vanka_omega=0.6)
    va = ce.vcycle(LEVEL, b)
    assert not np.array_equal(vg, va)
    # the coloured multiplicative smoother: captured and eager cycles agree
    for ctx in (cg, ce):
        ctx.set_params(smoother=1)
    vg2, ve2 = cg.vcycle(LEVEL, b), ce.vcycle(LEVEL, b)
    assert np.array_equal(vg2, ve2) and not np.array_equal(vg2, va)
    for ctx in (cg, ce):
        ctx.set_params(smoother=0)
    assert np.array_equal(cg.vcycle(LEVEL, b), va)
    for st in states:
        st.close()


def test_solves_and_steps_bitwise_equal_with_torch_stream():
    import torch
    stream = torch.cuda.Stream()
    cg, ce, lev = _pair(1, stream=stream.cuda_stream)
    n = lev[LEVEL].n_nodes
    # Newton steps from rest (the level-0 inverse is rebuilt every step)
    sg, se = cg.state(LEVEL), ce.state(LEVEL)
    for k in range(3):
        ig, ie = cg.step(sg, DT), ce.step(se, DT)
        print(f"[graphs] step {k}: {ig}", flush=True)
        xg, xe = sg.get()[0], se.get()[0]
        assert ig == ie
        assert np.array_equal(xg, xe), (k, np.abs(xg - xe).max())
    # GMRES solves on the linearisation at the last state
    for ctx, st in ((cg, sg), (ce, se)):
        ctx.linearize(st, LEVEL, DT)
    for rep in range(2):
        b = _rhs(lev, LEVEL, 70 + rep)
        (wg, ig), (we, ie) = cg.solve(LEVEL, b), ce.solve(LEVEL, b)
        assert ig == ie
        assert np.array_equal(wg, we)
    sg.close()
    se.close()
    assert n > 0


def test_autotuned_launches_are_bitwise_equal():
    import paper_2106_07687_amd as P
    macro = channel_obstacle(1)
    ctxs = []
    for tune in (1, 0):
        ctx = P.Context(precision=1, nu=macro.nu, autotune=tune)
        ctx.setup_mesh(macro, LEVEL)
        ctxs.append(ctx)
    for l in range(LEVEL + 1):
        cfg = ctxs[0].launch_config(l)
        print(f"[tune] level {l}: {cfg}", flush=True)
        assert set(cfg.values()) <= {0, 4, 16, 64, 128, 256, 1024}
        assert set(ctxs[1].launch_config(l).values()) <= {0, 256}
    sts = [c.state(LEVEL) for c in ctxs]
    for k in range(2):
        infos = [c.step(st, DT) for c, st in zip(ctxs, sts)]
        assert infos[0] == infos[1]
        assert np.array_equal(sts[0].get()[0], sts[1].get()[0]), k
    for st in sts:
        st.close()


def test_fused_residual_and_apply_is_bitwise_equal():
    """autotune=2 fuses the residual into the Vanka apply (sixteen lanes per
    cell), runs the SpMV with four threads per row on every level and fuses
    each coarse level's last update into the prolongation above it."""
    import paper_2106_07687_amd as P
    macro = channel_obstacle(2)
    ctxs = []
    for tune in (2, 0):
        ctx = P.Context(precision=1, nu=macro.nu, autotune=tune)
        ctx.setup_mesh(macro, LEVEL)
        ctxs.append(ctx)
    assert all(ctxs[0].launch_config(l)["vanka_smooth"] == 256 for l in range(1, LEVEL + 1))
    assert all(ctxs[0].launch_config(l)["spmv4"] == 256 for l in range(LEVEL + 1))
    assert all(ctxs[0].launch_config(l)["smooth_lanes"] == 16 for l in range(1, LEVEL + 1))
    assert [ctxs[0].launch_config(l)["update_prolong"] for l in range(LEVEL + 1)] == [0, 0] + [256] * (LEVEL - 1)
    assert all(ctxs[1].launch_config(l)["update_prolong"] == 0 for l in range(LEVEL + 1))
    assert all(ctxs[0].launch_config(l)["vanka_apply4"] == 256 for l in range(1, LEVEL + 1))
    assert all(ctxs[0].launch_config(l)["update_ordered"] == 256 for l in range(LEVEL + 1))
    lev = mesh.hierarchy(macro, LEVEL)
    x = random_state(lev[LEVEL].n_nodes, 5) * 0.3
    sts = []
    for ctx in ctxs:
        st = ctx.state(LEVEL)
        st.set(x, 0.0)
        ctx.linearize(st, LEVEL, DT)
        sts.append(st)
    for l in (LEVEL, 2, 1):
        b = _rhs(lev, l, 80 + l)
        x0 = _rhs(lev, l, 90 + l) * 0.1
        assert np.array_equal(ctxs[0].vanka_sweep(l, x0, b), ctxs[1].vanka_sweep(l, x0, b)), l
        assert np.array_equal(ctxs[0].vcycle(l, b), ctxs[1].vcycle(l, b)), l
    for st in sts:
        st.close()


def test_single_workgroup_bottom_cycle_is_bitwise_equal():
    """autotune=3 runs levels 1-2 and the coarse solve in one workgroup."""
    import paper_2106_07687_amd as P
    macro = channel_obstacle(3)
    ctxs = []
    for tune in (3, 0):
        ctx = P.Context(precision=1, nu=macro.nu, autotune=tune)
        ctx.setup_mesh(macro, LEVEL)
        ctxs.append(ctx)
    assert [ctxs[0].launch_config(l)["vcycle_small"] for l in range(LEVEL + 1)] == [0, 1024, 1024, 0]
    sts = [c.state(LEVEL) for c in ctxs]
    lev = mesh.hierarchy(macro, LEVEL)
    for k in range(2):
        infos = [c.step(st, DT) for c, st in zip(ctxs, sts)]
        assert infos[0] == infos[1], k
        assert np.array_equal(sts[0].get()[0], sts[1].get()[0]), k
    for l in (1, 2, LEVEL):
        b = _rhs(lev, l, 100 + l)
        assert np.array_equal(ctxs[0].vcycle(l, b), ctxs[1].vcycle(l, b)), l
    for st in sts:
        st.close()
